// Preconditioner apply P^-1 v = alpha D^-1 alpha^T v (Eq. 23, 24 and 28):
//
//  forward   y_j = v_j + sum_{k < j, j in S_k} alpha_kj^T y_k   (k ascending)
//            zt_j = D_j^-1 y_j
//  backward  z_k = zt_k + sum_{j in S_k} alpha_kj z_j             (k descending)
//
// Each sweep is one launch. A workgroup takes block rows by ticket (in the
// dependency order, so every row it waits for belongs to a workgroup that is
// already running) and its four wavefronts share the row's entries. A wave
// checks the ready flags of up to 64 of its entries at once with relaxed
// agent-scope loads, issues one acquire fence for the whole ready batch and
// processes it without workgroup barriers; it only spins on an entry that is
// not ready yet. Row results are published with a release fence and a flag
// store; the D^-1 product of the forward sweep comes after the flag, off the
// dependency chain.
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

}  // namespace

// Forward sweep; S right-hand sides per pass over a block.
template <int S>
__global__ void __launch_bounds__(NT)
k_sweep_fwd(int nb, const int64_t* __restrict__ blk_start, const int32_t* __restrict__ blk_size,
            const int64_t* __restrict__ colptr, const SweepEnt* __restrict__ colent, const cd* __restrict__ alpha,
            const cd* __restrict__ dinv, const int64_t* __restrict__ dinv_off, const cd* __restrict__ v,
            cd* __restrict__ yw, cd* __restrict__ zt, int64_t n, int nrhs, int* flags, unsigned long long* ctr,
            unsigned long long base, int epoch) {
    __shared__ int s_t;
    __shared__ cd part[NW][kMaxLeaf * S];
    __shared__ cd ysh[kMaxLeaf * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (;;) {
        const int j = take_ticket(ctr, base, &s_t);
        if (j >= nb) return;
        const int bj = blk_size[j];
        const int64_t sj = blk_start[j];
        const int64_t e0 = colptr[j];
        const int cnt = (int)(colptr[j + 1] - e0);
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            for_ready_entries(colent, e0, 1, cnt, flags, epoch, [&](const SweepEnt& e) {
                const int k = e.k, bk = blk_size[k];
                const int64_t sk = blk_start[k];
                cd y[2][S];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        const int a = lane + q * kWave;
                        y[q][c] = (a < bk && c < cs) ? yw[sk + a + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
                    }
                const cd* A = alpha + e.off;
                if (e.rank < 0) {
                    // out[b] += sum_a A[a][b] y_k[a]; RB rows of A loaded before use
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
                    // alpha = U V: out += V^T (U^T y_k); RB rank terms loaded at once
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
                    ysh[q] = s;
                    yw[sj + q % bj + (int64_t)(c0 + q / bj) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flags + j, epoch);
            }
            __syncthreads();
            // zt_j = D_j^-1 y_j, off the dependency chain: rows a = wid + NW r
            const cd* Di = dinv + dinv_off[j];
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
                        if (c >= cs) continue;
                        cd s = cmk(0.0, 0.0);
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int b = lane + q * kWave;
                            if (b < bj) s = cfma(Dr[r][q], ysh[b + c * bj], s);
                        }
                        s = wave_sum(s);
                        if (lane == 0) zt[sj + a + (int64_t)(c0 + c) * n] = s;
                    }
                }
            }
        }
    }
}

// Backward sweep; S right-hand sides per pass.
template <int S>
__global__ void __launch_bounds__(NT)
k_sweep_bwd(int nb, const int64_t* __restrict__ blk_start, const int32_t* __restrict__ blk_size,
            const int64_t* __restrict__ rowptr, const SweepEnt* __restrict__ rowent, const cd* __restrict__ alpha,
            const cd* __restrict__ zt, cd* __restrict__ z, int64_t n, int nrhs, int* flags, unsigned long long* ctr,
            unsigned long long base, int epoch) {
    __shared__ int s_t;
    __shared__ cd part[NW][kMaxLeaf * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (;;) {
        const int t = take_ticket(ctr, base, &s_t);
        if (t >= nb) return;
        const int k = nb - 1 - t;
        const int bk = blk_size[k];
        const int64_t sk = blk_start[k];
        const int64_t e_last = rowptr[k + 1] - 1;
        const int cnt = (int)(rowptr[k + 1] - rowptr[k]);
        for (int c0 = 0; c0 < nrhs; c0 += S) {
            const int cs = min(S, nrhs - c0);
            cd acc[2][S];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[q][c] = cmk(0.0, 0.0);
            // entries in descending j: the nearest block (usually the last to finish) comes last
            for_ready_entries(rowent, e_last, -1, cnt, flags, epoch, [&](const SweepEnt& e) {
                const int j = e.k, bj = blk_size[j];
                const int64_t sj = blk_start[j];
                cd zz[2][S];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        const int b = lane + q * kWave;
                        zz[q][c] = (b < bj && c < cs) ? z[sj + b + (int64_t)(c0 + c) * n] : cmk(0.0, 0.0);
                    }
                const cd* A = alpha + e.off;
                if (e.rank < 0) {
                    // acc[a] += sum_b A[a][b] z_j[b]: row sums across the wave, RB rows loaded at once
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
                    // alpha = U V: acc += U (V z_j); RB rank terms loaded at once
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
                    cd s = zt[sk + q % bk + (int64_t)(c0 + q / bk) * n];
#pragma unroll
                    for (int w = 0; w < NW; ++w) s = cadd(s, part[w][q]);
                    z[sk + q % bk + (int64_t)(c0 + q / bk) * n] = s;
                }
                if (c0 + S >= nrhs) publish(flags + k, epoch);
            }
            __syncthreads();
        }
    }
}

int sweep_grid(int64_t nb) { return (int)(nb < 1024 ? nb : 1024); }

void launch_sweeps(int64_t nb, const int64_t* blk_start, const int32_t* blk_size, const int64_t* colptr,
                   const SweepEnt* colent, const int64_t* rowptr, const SweepEnt* rowent, const cd* alpha,
                   const cd* dinv, const int64_t* dinv_off, const cd* v, cd* ywork, cd* z, int64_t n, int nrhs,
                   int* flags, unsigned long long* tickets, int epoch, hipStream_t s) {
    const int G = sweep_grid(nb);
    const unsigned long long base = (unsigned long long)(epoch - 1) * (unsigned long long)(nb + G);
    // flags: [0, nb) forward, [nb, 2 nb) backward; tickets[0] forward, tickets[1] backward
    const cd* ztc = ywork + n * nrhs;
    if (nrhs == 1) {
        hipLaunchKernelGGL(k_sweep_fwd<1>, dim3(G), dim3(NT), 0, s, (int)nb, blk_start, blk_size, colptr, colent, alpha,
                           dinv, dinv_off, v, ywork, ywork + n * nrhs, n, nrhs, flags, tickets, base, epoch);
        hipLaunchKernelGGL(k_sweep_bwd<1>, dim3(G), dim3(NT), 0, s, (int)nb, blk_start, blk_size, rowptr, rowent, alpha,
                           ztc, z, n, nrhs, flags + nb, tickets + 1, base, epoch);
    } else {
        hipLaunchKernelGGL(k_sweep_fwd<4>, dim3(G), dim3(NT), 0, s, (int)nb, blk_start, blk_size, colptr, colent, alpha,
                           dinv, dinv_off, v, ywork, ywork + n * nrhs, n, nrhs, flags, tickets, base, epoch);
        hipLaunchKernelGGL(k_sweep_bwd<4>, dim3(G), dim3(NT), 0, s, (int)nb, blk_start, blk_size, rowptr, rowent, alpha,
                           ztc, z, n, nrhs, flags + nb, tickets + 1, base, epoch);
    }
}

}  // namespace hs
