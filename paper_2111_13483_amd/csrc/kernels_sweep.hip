// Preconditioner apply P^-1 v = alpha D^-1 alpha^T v (Eq. 23, 24 and 28):
//
//  forward   y_j = v_j + sum_{k < j, j in S_k} alpha_kj^T y_k   (k ascending)
//            zt_j = D_j^-1 y_j
//  backward  z_k = zt_k + sum_{j in S_k} alpha_kj z_j             (k descending)
//
// Under a bandwidth-reducing order each block row depends on the one before
// it, so both sweeps are chains of nb dependent steps. Consecutive rows are
// grouped into chunks and the in-chunk coupling is applied through the
// explicit inverse Linv of the chunk's unit lower-triangular factor
// (forward: y_c = Linv_c r_c; backward: z_c = Linv_c^T r'_c), where r
// collects the cross-chunk terms. The chain then advances a chunk at a time:
// phase A of a row gathers its cross-chunk entries, phase B applies its rows
// (forward) or columns (backward) of Linv once every row of the chunk has
// finished phase A. The operator is unchanged; only the evaluation order of
// the triangular solves differs.
//
// Each sweep is one launch. A workgroup takes block rows by ticket in the
// dependency order, so every row it waits for belongs to a workgroup that is
// already running. A wave checks the ready flags of up to 64 entries at once
// with relaxed agent-scope loads, takes one acquire fence per ready batch and
// spins only on an entry that is not ready yet. Results are published with a
// release fence and a flag store; D^-1 follows the forward flag, off the
// chain.
#include "devcommon.h"
#include "kernels.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;
constexpr int RB = 8;    // block rows (or rank terms) whose loads are issued together

__device__ __forceinline__ int relaxed_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ cd shfl_cd(cd v, int src) {
    return cmk(__shfl(v.x, src, kWave), __shfl(v.y, src, kWave));
}

__device__ __forceinline__ int take_ticket(unsigned long long* ctr, unsigned long long base, int* s_t) {
    __syncthreads();
    if (threadIdx.x == 0) *s_t = (int)(atomicAdd(ctr, 1ull) - base);
    __syncthreads();
    return *s_t;
}

// Publish a row: wave-local stores are complete and visible agent-wide
// before the flag.
__device__ __forceinline__ void publish(int* flag, int epoch) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x % kWave) == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Walk this wave's entries (positions w, w + NW, ... of [0, cnt) in the
// list `ent` starting at `e0` with step `dir`), waiting for each entry's
// block to be ready, and call body(entry) in list order.
template <class Body>
__device__ __forceinline__ void for_ready_entries(const SweepEnt* __restrict__ ents, int64_t e0, int dir, int cnt,
                                                  const int* flags, int epoch, Body body) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int mine = cnt > wid ? (cnt - wid + NW - 1) / NW : 0;
    for (int qb = 0; qb < mine; qb += kWave) {
        const int nv = min(kWave, mine - qb);
        SweepEnt my{};
        if (lane < nv) my = ents[e0 + (int64_t)dir * (wid + NW * (qb + lane))];
        int done = 0;
        while (done < nv) {
            const bool pending = lane >= done && lane < nv;
            const bool ok = !pending || relaxed_load(flags + my.k) == epoch;
            const unsigned long long m = __ballot(ok);
            // first lane at or after `done` that is not ready
            const unsigned long long notready = ~m & (nv == kWave ? ~0ull : ((1ull << nv) - 1ull));
            const int upto = notready ? __builtin_ctzll(notready) : nv;
            if (upto <= done) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int p = done; p < upto; ++p) {
                SweepEnt e;
                e.off = __shfl(my.off, p, kWave);
                e.k = __shfl(my.k, p, kWave);
                e.rank = __shfl(my.rank, p, kWave);
                body(e);
            }
            done = upto;
        }
    }
}
// Wait until flags[first..last] all equal epoch (whole wave), then acquire.
__device__ __forceinline__ void wait_range(const int* flags, int first, int last, int epoch) {
    const int lane = threadIdx.x % kWave;
    for (int b0 = first; b0 <= last; b0 += kWave) {
        const int f = b0 + lane;
        for (;;) {
            const bool ok = f > last || relaxed_load(flags + f) == epoch;
            if (__ballot(!ok) == 0ull) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

constexpr int QC = kMaxChunk / kWave;   // 64-wide column groups of a chunk
constexpr int RB2 = 4;                  // Linv rows whose loads are issued together

}  // namespace

// Forward sweep; S right-hand sides per pass.
template <int S>
__global__ void __launch_bounds__(NT)
k_sweep_fwd(SweepPlan p, const cd* __restrict__ v, SweepWork wk, int nrhs, unsigned long long base, int epoch) {
    __shared__ int s_t;
    __shared__ cd part[NW][kMaxLeaf * S];
    __shared__ cd ysh[kMaxLeaf * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t n = p.n;
    int* flagY = wk.flags;
    int* flagR = wk.flags + p.nb;
    for (;;) {
        const int j = take_ticket(wk.tickets, base, &s_t);
        if (j >= p.nb) return;
        const int bj = p.bsize[j];
        const int64_t sj = p.bstart[j];
        const int64_t e0 = p.colptr[j];
        const int cnt = (int)(p.colptr[j + 1] - e0);
        // ---- phase A: r_j = v_j + cross-chunk terms
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            for_ready_entries(p.colent, e0, 1, cnt, flagY, epoch, [&](const SweepEnt& e) {
                const int k = e.k, bk = p.bsize[k];
                const int64_t sk = p.bstart[k];
                cd y[2][S];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        const int a = lane + q * kWave;
                        y[q][c] = (a < bk && c < cs) ? wk.yw[sk + a + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
                    }
                const cd* A = p.alpha + e.off;
                if (e.rank < 0) {
                    for (int a0 = 0; a0 < bk; a0 += RB) {
                        cd Ar[RB][2];
#pragma unroll
                        for (int r = 0; r < RB; ++r)
#pragma unroll
                            for (int q = 0; q < 2; ++q) {
                                const int b = lane + q * kWave;
                                Ar[r][q] = (a0 + r < bk && b < bj) ? A[(int64_t)(a0 + r) * bj + b] : cmk(0.0, 0.0);
                            }
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            const int a = a0 + r;
                            if (a < bk)
#pragma unroll
                            for (int c = 0; c < S; ++c) {
                                const cd ya = shfl_cd(a < kWave ? y[0][c] : y[1][c], a % kWave);
#pragma unroll
                                for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Ar[r][q], ya, acc[q][c]);
                            }
                        }
                    }
                } else {
                    const int rk = e.rank;
                    const cd* Uf = A;
                    const cd* Vf = A + (int64_t)bk * rk;
                    for (int l0 = 0; l0 < rk; l0 += RB) {
                        cd Ur[RB][2], Vr[RB][2];
#pragma unroll
                        for (int r = 0; r < RB; ++r)
#pragma unroll
                            for (int q = 0; q < 2; ++q) {
                                const int x = lane + q * kWave;
                                const bool on = l0 + r < rk;
                                Ur[r][q] = (on && x < bk) ? Uf[(int64_t)(l0 + r) * bk + x] : cmk(0.0, 0.0);
                                Vr[r][q] = (on && x < bj) ? Vf[(int64_t)(l0 + r) * bj + x] : cmk(0.0, 0.0);
                            }
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            if (l0 + r < rk)
#pragma unroll
                            for (int c = 0; c < S; ++c) {
                                cd t = cmul(Ur[r][0], y[0][c]);
                                t = cfma(Ur[r][1], y[1][c], t);
                                t = wave_sum(t);
#pragma unroll
                                for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Vr[r][q], t, acc[q][c]);
                            }
                        }
                    }
                }
            });
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int b = lane + q * kWave;
                if (b < bj)
#pragma unroll
                    for (int c = 0; c < S; ++c)
                        if (c < cs) part[wid][b + c * bj] = acc[q][c];
            }
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < bj * cs; q += kWave) {
                    cd s = v[sj + q % bj + (int64_t)(c0 + q / bj) * n];
#pragma unroll
                    for (int w = 0; w < NW; ++w) s = cadd(s, part[w][q]);
                    wk.rbuf[p.pos[j] + q % bj + (int64_t)(c0 + q / bj) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flagR + j, epoch);
            }
            __syncthreads();
        }
        // ---- phase B: y_j = rows of Linv_c times r_c
        const int cf = p.cfirst[j];
        const int wj = p.w[j];
        const int64_t pc = p.pos[cf];
        const cd* X = p.linv + p.linv_off[j];
        wait_range(flagR, cf, j, epoch);
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd rr[QC][S];
#pragma unroll
            for (int q = 0; q < QC; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const int col = lane + q * kWave;
                    rr[q][c] = (col < wj && c < cs) ? wk.rbuf[pc + col + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
                }
            for (int a0 = wid; a0 < bj; a0 += NW * RB2) {
                cd Xr[RB2][QC];
#pragma unroll
                for (int r = 0; r < RB2; ++r)
#pragma unroll
                    for (int q = 0; q < QC; ++q) {
                        const int a = a0 + NW * r, col = lane + q * kWave;
                        Xr[r][q] = (a < bj && col < wj) ? X[(int64_t)a * wj + col] : cmk(0.0, 0.0);
                    }
#pragma unroll
                for (int r = 0; r < RB2; ++r) {
                    const int a = a0 + NW * r;
                    if (a < bj)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        cd sacc = cmk(0.0, 0.0);
#pragma unroll
                        for (int q = 0; q < QC; ++q) sacc = cfma(Xr[r][q], rr[q][c], sacc);
                        sacc = wave_sum(sacc);
                        if (lane == 0 && c < cs) wk.yw[sj + a + (int64_t)(c0 + c) * n] = sacc;
                    }
                }
            }
        }
        __syncthreads();
        if (wid == 0) publish(flagY + j, epoch);
        // ---- zt_j = D_j^-1 y_j, off the chain
        const cd* Di = p.dinv + p.dinv_off[j];
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            for (int q = tid; q < bj * cs; q += NT) ysh[q] = wk.yw[sj + q % bj + (int64_t)(c0 + q / bj) * n];
            __syncthreads();
            for (int a0 = wid; a0 < bj; a0 += NW * RB) {
                cd Dr[RB][2];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int a = a0 + NW * r, b = lane + q * kWave;
                        Dr[r][q] = (a < bj && b < bj) ? Di[(int64_t)a * bj + b] : cmk(0.0, 0.0);
                    }
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int a = a0 + NW * r;
                    if (a < bj)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        cd sacc = cmk(0.0, 0.0);
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int b = lane + q * kWave;
                            if (b < bj) sacc = cfma(Dr[r][q], ysh[b + c * bj], sacc);
                        }
                        sacc = wave_sum(sacc);
                        if (lane == 0 && c < cs) wk.zt[sj + a + (int64_t)(c0 + c) * n] = sacc;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Backward sweep; S right-hand sides per pass.
template <int S>
__global__ void __launch_bounds__(NT)
k_sweep_bwd(SweepPlan p, cd* __restrict__ z, SweepWork wk, int nrhs, unsigned long long base, int epoch) {
    __shared__ int s_t;
    __shared__ cd part[NW][kMaxLeaf * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t n = p.n;
    int* flagZ = wk.flags + 2 * p.nb;
    int* flagR = wk.flags + 3 * p.nb;
    for (;;) {
        const int t = take_ticket(wk.tickets + 1, base, &s_t);
        if (t >= p.nb) return;
        const int k = p.nb - 1 - t;
        const int bk = p.bsize[k];
        const int64_t sk = p.bstart[k];
        const int64_t e_last = p.rowptr[k + 1] - 1;
        const int cnt = (int)(p.rowptr[k + 1] - p.rowptr[k]);
        // ---- phase A: r'_k = zt_k + cross-chunk terms (j descending: the nearest comes last)
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            for_ready_entries(p.rowent, e_last, -1, cnt, flagZ, epoch, [&](const SweepEnt& e) {
                const int j = e.k, bj = p.bsize[j];
                const int64_t sj = p.bstart[j];
                cd zz[2][S];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        const int b = lane + q * kWave;
                        zz[q][c] = (b < bj && c < cs) ? z[sj + b + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
                    }
                const cd* A = p.alpha + e.off;
                if (e.rank < 0) {
                    for (int a0 = 0; a0 < bk; a0 += RB) {
                        cd Ar[RB][2];
#pragma unroll
                        for (int r = 0; r < RB; ++r)
#pragma unroll
                            for (int q = 0; q < 2; ++q) {
                                const int b = lane + q * kWave;
                                Ar[r][q] = (a0 + r < bk && b < bj) ? A[(int64_t)(a0 + r) * bj + b] : cmk(0.0, 0.0);
                            }
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            const int a = a0 + r;
                            if (a < bk)
#pragma unroll
                            for (int c = 0; c < S; ++c) {
                                cd sr = cmul(Ar[r][0], zz[0][c]);
                                sr = cfma(Ar[r][1], zz[1][c], sr);
                                sr = wave_sum(sr);
                                if (lane == a % kWave) {
                                    if (a < kWave) acc[0][c] = cadd(acc[0][c], sr);
                                    else acc[1][c] = cadd(acc[1][c], sr);
                                }
                            }
                        }
                    }
                } else {
                    const int rk = e.rank;
                    const cd* Uf = A;
                    const cd* Vf = A + (int64_t)bk * rk;
                    for (int l0 = 0; l0 < rk; l0 += RB) {
                        cd Ur[RB][2], Vr[RB][2];
#pragma unroll
                        for (int r = 0; r < RB; ++r)
#pragma unroll
                            for (int q = 0; q < 2; ++q) {
                                const int x = lane + q * kWave;
                                const bool on = l0 + r < rk;
                                Ur[r][q] = (on && x < bk) ? Uf[(int64_t)(l0 + r) * bk + x] : cmk(0.0, 0.0);
                                Vr[r][q] = (on && x < bj) ? Vf[(int64_t)(l0 + r) * bj + x] : cmk(0.0, 0.0);
                            }
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            if (l0 + r < rk)
#pragma unroll
                            for (int c = 0; c < S; ++c) {
                                cd tt = cmul(Vr[r][0], zz[0][c]);
                                tt = cfma(Vr[r][1], zz[1][c], tt);
                                tt = wave_sum(tt);
#pragma unroll
                                for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Ur[r][q], tt, acc[q][c]);
                            }
                        }
                    }
                }
            });
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int a = lane + q * kWave;
                if (a < bk)
#pragma unroll
                    for (int c = 0; c < S; ++c)
                        if (c < cs) part[wid][a + c * bk] = acc[q][c];
            }
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < bk * cs; q += kWave) {
                    cd s = wk.zt[sk + q % bk + (int64_t)(c0 + q / bk) * n];
#pragma unroll
                    for (int w = 0; w < NW; ++w) s = cadd(s, part[w][q]);
                    wk.rbuf2[p.pos[k] + q % bk + (int64_t)(c0 + q / bk) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flagR + k, epoch);
            }
            __syncthreads();
        }
        // ---- phase B: z_k = (columns of Linv_c for block k)^T r'_c
        const int cl = p.clast[k];
        const int lk = p.loc[k];
        wait_range(flagR, k, cl, epoch);
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            // wave w takes blocks k' = k + w, k + w + NW, ... of the chunk
            for (int kp = k + wid; kp <= cl; kp += NW) {
                const int bp = p.bsize[kp], wp = p.w[kp];
                const cd* X = p.linv + p.linv_off[kp];
                const int64_t rp = p.pos[kp];
                for (int b0 = 0; b0 < bp; b0 += RB) {
                    cd Xr[RB][2], rv[RB][S];
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int a = lane + q * kWave;
                            Xr[r][q] = (b0 + r < bp && a < bk) ? X[(int64_t)(b0 + r) * wp + lk + a] : cmk(0.0, 0.0);
                        }
#pragma unroll
                        for (int c = 0; c < S; ++c)
                            rv[r][c] = (b0 + r < bp && c < cs) ? wk.rbuf2[rp + b0 + r + (int64_t)(c0 + c) * n]
                                                               : cmk(0.0, 0.0);
                    }
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int q = 0; q < 2; ++q)
#pragma unroll
                            for (int c = 0; c < S; ++c) acc[q][c] = cfma(Xr[r][q], rv[r][c], acc[q][c]);
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int a = lane + q * kWave;
                if (a < bk)
#pragma unroll
                    for (int c = 0; c < S; ++c)
                        if (c < cs) part[wid][a + c * bk] = acc[q][c];
            }
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < bk * cs; q += kWave) {
                    cd s = part[0][q];
#pragma unroll
                    for (int w = 1; w < NW; ++w) s = cadd(s, part[w][q]);
                    z[sk + q % bk + (int64_t)(c0 + q / bk) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flagZ + k, epoch);
            }
            __syncthreads();
        }
    }
}

// Linv of each chunk (one workgroup per chunk), row blocks in order:
// X_j = E_j + sum_{in-chunk (k, j)} alpha_kj^T X_k, X_k stored b_k x w_k.
__global__ void __launch_bounds__(NT)
k_linv(SweepPlan p, const int32_t* __restrict__ chunk_first, const int64_t* __restrict__ intptr,
       const SweepEnt* __restrict__ intent, const cd* __restrict__ A, cd* __restrict__ linv) {
    const int c = blockIdx.x;
    const int j0 = chunk_first[c], j1 = chunk_first[c + 1];
    for (int j = j0; j < j1; ++j) {
        const int bj = p.bsize[j], wj = p.w[j], lj = p.loc[j];
        cd* X = linv + p.linv_off[j];
        for (int e = threadIdx.x; e < bj * wj; e += NT) {
            const int a = e / wj, col = e % wj;
            cd val = cmk(col == lj + a ? 1.0 : 0.0, 0.0);
            for (int64_t q = intptr[j]; q < intptr[j + 1]; ++q) {
                const SweepEnt en = intent[q];
                const int k = en.k, bk = p.bsize[k], wkk = p.w[k];
                if (col >= wkk) continue;
                const cd* Ak = A + en.off;
                const cd* Xk = linv + p.linv_off[k];
                for (int l = 0; l < bk; ++l) val = cfma(Ak[(int64_t)l * bj + a], Xk[(int64_t)l * wkk + col], val);
            }
            X[e] = val;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT)
k_lr_expand(const ExpandTask* __restrict__ tasks, const cd* __restrict__ src, cd* __restrict__ dst) {
    const ExpandTask t = tasks[blockIdx.x];
    const cd* U = src + t.src_off;
    const cd* V = U + (int64_t)t.m * t.r;
    cd* D = dst + t.dst_off;
    for (int e = threadIdx.x; e < t.m * t.n; e += NT) {
        const int a = e / t.n, b = e % t.n;
        cd s = cmk(0.0, 0.0);
        for (int l = 0; l < t.r; ++l) s = cfma(U[(int64_t)l * t.m + a], V[(int64_t)l * t.n + b], s);
        D[e] = s;
    }
}

int sweep_grid(int64_t nb) { return (int)(nb < 1024 ? nb : 1024); }

void launch_sweeps(const SweepPlan& p, const cd* v, cd* z, int nrhs, const SweepWork& w, int epoch, hipStream_t s) {
    const int G = sweep_grid(p.nb);
    const unsigned long long base = (unsigned long long)(epoch - 1) * (unsigned long long)(p.nb + G);
    if (nrhs == 1) {
        hipLaunchKernelGGL(k_sweep_fwd<1>, dim3(G), dim3(NT), 0, s, p, v, w, nrhs, base, epoch);
        hipLaunchKernelGGL(k_sweep_bwd<1>, dim3(G), dim3(NT), 0, s, p, z, w, nrhs, base, epoch);
    } else {
        hipLaunchKernelGGL(k_sweep_fwd<4>, dim3(G), dim3(NT), 0, s, p, v, w, nrhs, base, epoch);
        hipLaunchKernelGGL(k_sweep_bwd<4>, dim3(G), dim3(NT), 0, s, p, z, w, nrhs, base, epoch);
    }
}

void launch_linv(const SweepPlan& p, int nchunk, const int32_t* chunk_first, const int64_t* intptr,
                 const SweepEnt* intent, const cd* A, cd* linv, hipStream_t s) {
    if (nchunk > 0)
        hipLaunchKernelGGL(k_linv, dim3(nchunk), dim3(NT), 0, s, p, chunk_first, intptr, intent, A, linv);
}

void launch_lr_expand(const ExpandTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_lr_expand, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, src, dst);
}

}  // namespace hs
