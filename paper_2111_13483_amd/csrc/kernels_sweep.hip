// Preconditioner apply P^-1 v = alpha D^-1 alpha^T v (Eq. 23, 24 and 28):
//
//  forward   y_j = v_j + sum_{k < j, j in S_k} alpha_kj^T y_k   (k ascending)
//            zt_j = D_j^-1 y_j
//  backward  z_k = zt_k + sum_{j in S_k} alpha_kj z_j             (k descending)
//
// Under a bandwidth-reducing order each block row depends on the one before
// it, so both sweeps are chains of nb dependent steps. Consecutive rows are
// grouped into chunks; with Linv_c the explicit inverse of chunk c's unit
// lower-triangular diagonal part and C_c its coupling to chunk c-1,
//   forward   y_c = Linv_c r_c + (Linv_c C_c) y_{c-1}
//   backward  z_c = Linv_c^T r'_c + (Linv_c^T C_{c+1}^T) z_{c+1}
// where r, r' gather the terms from chunks two or more away. Phase A of a
// row gathers those terms (they are ready long before they are needed);
// phase B applies the row's slice of the two dense products once its chunk
// neighbour has finished, so the chain advances one dense row-block product
// per chunk. The operator is unchanged; only the evaluation order of the
// triangular solves differs.
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
// Wait until flags[first..last] all equal epoch (whole wave); no fence.
__device__ __forceinline__ void wait_range_nofence(const int* flags, int first, int last, int epoch) {
    const int lane = threadIdx.x % kWave;
    for (int b0 = first; b0 <= last; b0 += kWave) {
        const int f = b0 + lane;
        for (;;) {
            const bool ok = f > last || relaxed_load(flags + f) == epoch;
            if (__ballot(!ok) == 0ull) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

constexpr int QC = kMaxChunk / kWave;   // 64-wide column groups of a chunk
constexpr int RB2 = 2;                  // dense rows whose loads are issued together

// Phase A accumulation over one list of entries (forward: alpha^T y_k into
// columns b of the row block; backward: alpha z_j into rows a).
template <int S, bool FWD>
__device__ __forceinline__ void phase_a(const SweepPlan& p, const SweepEnt* ents, int64_t e0, int dir, int cnt,
                                        const int* flags, int epoch, const cd* src, int c0, int cs, int bme,
                                        cd (&acc)[2][S]) {
    const int lane = threadIdx.x % kWave;
    const int64_t n = p.n;
    for_ready_entries(ents, e0, dir, cnt, flags, epoch, [&](const SweepEnt& e) {
        const int o = e.k, bo = p.bsize[o];
        const int64_t so = p.pos[o];
        cd x[2][S];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < S; ++c) {
                const int a = lane + q * kWave;
                x[q][c] = (a < bo && c < cs) ? src[so + a + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
            }
        // the stored block is alpha_{row, col}: forward (row = o, col = me), backward (row = me, col = o)
        const int rows = FWD ? bo : bme, cols = FWD ? bme : bo;
        const cd* A = p.alpha + e.off;
        if (e.rank < 0) {
            for (int a0 = 0; a0 < rows; a0 += RB) {
                cd Ar[RB][2];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int b = lane + q * kWave;
                        Ar[r][q] = (a0 + r < rows && b < cols) ? A[(int64_t)(a0 + r) * cols + b] : cmk(0.0, 0.0);
                    }
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int a = a0 + r;
                    if (a < rows)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        if (FWD) {
                            const cd xa = shfl_cd(a < kWave ? x[0][c] : x[1][c], a % kWave);
#pragma unroll
                            for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Ar[r][q], xa, acc[q][c]);
                        } else {
                            cd sr = cmul(Ar[r][0], x[0][c]);
                            sr = cfma(Ar[r][1], x[1][c], sr);
                            sr = wave_sum(sr);
                            if (lane == a % kWave) {
                                if (a < kWave) acc[0][c] = cadd(acc[0][c], sr);
                                else acc[1][c] = cadd(acc[1][c], sr);
                            }
                        }
                    }
                }
            }
        } else {
            const int rk = e.rank;
            const cd* Uf = A;
            const cd* Vf = A + (int64_t)rows * rk;
            for (int l0 = 0; l0 < rk; l0 += RB) {
                cd Ur[RB][2], Vr[RB][2];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int xx = lane + q * kWave;
                        const bool on = l0 + r < rk;
                        Ur[r][q] = (on && xx < rows) ? Uf[(int64_t)(l0 + r) * rows + xx] : cmk(0.0, 0.0);
                        Vr[r][q] = (on && xx < cols) ? Vf[(int64_t)(l0 + r) * cols + xx] : cmk(0.0, 0.0);
                    }
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    if (l0 + r < rk)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        if (FWD) {   // out += V^T (U^T x)
                            cd t = cmul(Ur[r][0], x[0][c]);
                            t = cfma(Ur[r][1], x[1][c], t);
                            t = wave_sum(t);
#pragma unroll
                            for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Vr[r][q], t, acc[q][c]);
                        } else {     // out += U (V x)
                            cd t = cmul(Vr[r][0], x[0][c]);
                            t = cfma(Vr[r][1], x[1][c], t);
                            t = wave_sum(t);
#pragma unroll
                            for (int q = 0; q < 2; ++q) acc[q][c] = cfma(Ur[r][q], t, acc[q][c]);
                        }
                    }
                }
            }
        }
    });
}

// out rows a (wave-strided) of [A1 | A2] x [x1; x2]: A1 is rows x w1 at a1,
// x1 = src1[o1 + col]; A2 rows x w2 at a2, x2 = src2[o2 + col] (w2 may be 0).
template <int S>
__device__ __forceinline__ void dense_rows(const cd* A1, int w1, const cd* src1, int64_t o1, const cd* A2, int w2,
                                           const cd* src2, int64_t o2, int rows, int64_t n, int c0, int cs,
                                           cd* out_lds) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    cd x1[QC][S], x2[QC][S];
#pragma unroll
    for (int q = 0; q < QC; ++q)
#pragma unroll
        for (int c = 0; c < S; ++c) {
            const int col = lane + q * kWave;
            x1[q][c] = (col < w1 && c < cs) ? src1[o1 + col + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
            x2[q][c] = (col < w2 && c < cs) ? src2[o2 + col + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
        }
    for (int a0 = wid; a0 < rows; a0 += NW * RB2) {
        cd R1[RB2][QC], R2[RB2][QC];
#pragma unroll
        for (int r = 0; r < RB2; ++r)
#pragma unroll
            for (int q = 0; q < QC; ++q) {
                const int a = a0 + NW * r, col = lane + q * kWave;
                R1[r][q] = (a < rows && col < w1) ? A1[(int64_t)a * w1 + col] : cmk(0.0, 0.0);
                R2[r][q] = (a < rows && col < w2) ? A2[(int64_t)a * w2 + col] : cmk(0.0, 0.0);
            }
#pragma unroll
        for (int r = 0; r < RB2; ++r) {
            const int a = a0 + NW * r;
            if (a < rows)
#pragma unroll
            for (int c = 0; c < S; ++c) {
                cd sacc = cmk(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    sacc = cfma(R1[r][q], x1[q][c], sacc);
                    sacc = cfma(R2[r][q], x2[q][c], sacc);
                }
                sacc = wave_sum(sacc);
                if (lane == 0 && c < cs) out_lds[a + c * rows] = sacc;
            }
        }
    }
}

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
        const int64_t sj = p.bstart[j], pj = p.pos[j];
        const int64_t e0 = p.colptr[j];
        const int cnt = (int)(p.colptr[j + 1] - e0);
        // ---- phase A: r_j = v_j + terms from chunks two or more back
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            phase_a<S, true>(p, p.colent, e0, 1, cnt, flagY, epoch, wk.ybuf, c0, cs, bj, acc);
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
                    wk.rbuf[pj + q % bj + (int64_t)(c0 + q / bj) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flagR + j, epoch);
            }
            __syncthreads();
        }
        // ---- phase B: y_j = Linv rows r_c + (Linv C) rows y_{c-1}
        const int cf = p.cfirst[j];
        const int pf = p.pf[j], pl = p.pl[j];
        wait_range_nofence(flagR, cf, j, epoch);
        if (pf >= 0) wait_range_nofence(flagY, pf, pl, epoch);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int wprev = pf >= 0 ? (int)(p.pos[pl] + p.bsize[pl] - p.pos[pf]) : 0;
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            dense_rows<S>(p.lf + p.lf_off[j], p.w[j], wk.rbuf, p.pos[cf], p.mf + p.mf_off[j], wprev, wk.ybuf,
                          pf >= 0 ? p.pos[pf] : 0, bj, n, c0, cs, ysh);
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < bj * cs; q += kWave)
                    wk.ybuf[pj + q % bj + (int64_t)(c0 + q / bj) * n] = ysh[q];
                if (c0 + S >= nrhs) publish(flagY + j, epoch);
            }
            __syncthreads();
            // zt_j = D_j^-1 y_j, off the chain
            const cd* Di = p.dinv + p.dinv_off[j];
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
    __shared__ cd zsh[kMaxLeaf * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t n = p.n;
    int* flagZ = wk.flags + 2 * p.nb;
    int* flagR = wk.flags + 3 * p.nb;
    for (;;) {
        const int t = take_ticket(wk.tickets + 1, base, &s_t);
        if (t >= p.nb) return;
        const int k = p.nb - 1 - t;
        const int bk = p.bsize[k];
        const int64_t sk = p.bstart[k], pk = p.pos[k];
        const int64_t e_last = p.rowptr[k + 1] - 1;
        const int cnt = (int)(p.rowptr[k + 1] - p.rowptr[k]);
        // ---- phase A: r'_k = zt_k + terms from chunks two or more ahead (nearest last)
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            phase_a<S, false>(p, p.rowent, e_last, -1, cnt, flagZ, epoch, wk.zbuf, c0, cs, bk, acc);
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
                    wk.rbuf2[pk + q % bk + (int64_t)(c0 + q / bk) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flagR + k, epoch);
            }
            __syncthreads();
        }
        // ---- phase B: z_k = Linv^T rows r'_c + (Linv^T C^T) rows z_{c+1}
        const int cl = p.clast[k];
        const int nf = p.nf[k], nl = p.nl[k];
        wait_range_nofence(flagR, k, cl, epoch);
        if (nf >= 0) wait_range_nofence(flagZ, nf, nl, epoch);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int wnext = nf >= 0 ? (int)(p.pos[nl] + p.bsize[nl] - p.pos[nf]) : 0;
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            dense_rows<S>(p.lb + p.lb_off[k], p.wt[k], wk.rbuf2, pk, p.mb + p.mb_off[k], wnext, wk.zbuf,
                          nf >= 0 ? p.pos[nf] : 0, bk, n, c0, cs, zsh);
            __syncthreads();
            if (wid == 0) {
                for (int q = lane; q < bk * cs; q += kWave) {
                    wk.zbuf[pk + q % bk + (int64_t)(c0 + q / bk) * n] = zsh[q];
                    z[sk + q % bk + (int64_t)(c0 + q / bk) * n] = zsh[q];
                }
                if (c0 + S >= nrhs) publish(flagZ + k, epoch);
            }
            __syncthreads();
        }
    }
}

// Linv rows of each chunk (one workgroup per chunk), row blocks in order:
// X_j = E_j + sum_{in-chunk (k, j)} alpha_kj^T X_k, X_k stored b_k x w_k.
__global__ void __launch_bounds__(NT)
k_linv(SweepPlan p, const int32_t* __restrict__ chunk_first, const int64_t* __restrict__ intptr,
       const SweepEnt* __restrict__ intent, const cd* __restrict__ A, cd* __restrict__ lf) {
    const int c = blockIdx.x;
    const int j0 = chunk_first[c], j1 = chunk_first[c + 1];
    for (int j = j0; j < j1; ++j) {
        const int bj = p.bsize[j], wj = p.w[j], lj = p.loc[j];
        cd* X = lf + p.lf_off[j];
        for (int e = threadIdx.x; e < bj * wj; e += NT) {
            const int a = e / wj, col = e % wj;
            cd val = cmk(col == lj + a ? 1.0 : 0.0, 0.0);
            for (int64_t q = intptr[j]; q < intptr[j + 1]; ++q) {
                const SweepEnt en = intent[q];
                const int k = en.k, bk = p.bsize[k], wkk = p.w[k];
                if (col >= wkk) continue;
                const cd* Ak = A + en.off;
                const cd* Xk = lf + p.lf_off[k];
                for (int l = 0; l < bk; ++l) val = cfma(Ak[(int64_t)l * bj + a], Xk[(int64_t)l * wkk + col], val);
            }
            X[e] = val;
        }
        __syncthreads();
    }
}

// Linv^T row block k: LT_k[a][col] = Linv[loc_k + col][loc_k + a], col < wt_k.
__global__ void __launch_bounds__(NT)
k_linv_transpose(SweepPlan p, cd* __restrict__ lb) {
    const int k = blockIdx.x;
    const int bk = p.bsize[k], wtk = p.wt[k], lk = p.loc[k];
    const int cl = p.clast[k];
    cd* out = lb + p.lb_off[k];
    for (int e = threadIdx.x; e < bk * wtk; e += NT) {
        const int a = e / wtk, col = e % wtk;
        const int row = lk + col;          // chunk row index
        // find the block kp holding chunk row `row` (blocks k..cl)
        int kp = k;
        while (kp < cl && p.loc[kp] + p.bsize[kp] <= row) ++kp;
        const int rr = row - p.loc[kp];
        const int wkp = p.w[kp];
        const int cc = lk + a;
        out[e] = cc < wkp ? p.lf[p.lf_off[kp] + (int64_t)rr * wkp + cc] : cmk(0.0, 0.0);
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
                 const SweepEnt* intent, const cd* A, cd* lf, hipStream_t s) {
    if (nchunk > 0)
        hipLaunchKernelGGL(k_linv, dim3(nchunk), dim3(NT), 0, s, p, chunk_first, intptr, intent, A, lf);
}

void launch_linv_transpose(const SweepPlan& p, cd* lb, hipStream_t s) {
    if (p.nb > 0) hipLaunchKernelGGL(k_linv_transpose, dim3(p.nb), dim3(NT), 0, s, p, lb);
}

void launch_lr_expand(const ExpandTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_lr_expand, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, src, dst);
}

}  // namespace hs
