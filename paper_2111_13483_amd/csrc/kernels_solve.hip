// gfx950 kernels of the solve phase:
//  * H-matrix matvec Z x = Z_N x + Z_F x (Eq. 11): each stored near block
//    is read once and applied as Z_ij x_j and Z_ij^T x_i; each far block
//    gives U (V x_s) and V^T (U^T x_t); per-block results go to private
//    slots and a per-leaf gather sums them in a fixed order (deterministic);
//  * right-preconditioned GMRES building blocks with per-column state:
//    classical Gram-Schmidt twice, complex Givens rotations, restart.
#include "devcommon.h"
#include "kernels.h"

namespace hs {

namespace {
constexpr int NT = 256;
constexpr int NW = NT / kWave;
constexpr int SCH = 4;   // right-hand sides per pass over a block
}

// ---------------------------------------------------------------- permute
__global__ void k_permute(const cd* __restrict__ src, cd* __restrict__ dst, const int64_t* __restrict__ perm, int64_t n,
                          int64_t nrhs, int to_tree) {
    const int64_t tot = n * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, c = e / n;
        if (to_tree) dst[e] = src[perm[i] + c * n];
        else dst[perm[i] + c * n] = src[e];
    }
}

// ---------------------------------------------------------------- near matvec
// One workgroup per stored near block Z_ij (m x nn, row-major): s1 = Z_ij x_j
// (rows, one wave per row, RU rows' loads issued together) and, off the
// diagonal, s2 = Z_ij^T x_i (columns, lanes over columns, then the waves'
// partial sums in a fixed order). S right-hand sides per pass.
template <int S, class T>
__global__ void __launch_bounds__(NT)
k_near_mv(ColMask mk, const NearTask* __restrict__ tasks, const int64_t* __restrict__ slot_base, const T* __restrict__ Z,
          const cd* __restrict__ x, int64_t n, int nrhs, cd* __restrict__ slots) {
    using A = arith_t<T>;
    constexpr int RU = 4;
    __shared__ A xi[kMaxLeaf * S], xj[kMaxLeaf * S];
    __shared__ A colp[NW][kMaxLeaf * S];
    const NearTask t = tasks[blockIdx.x];
    const int m = t.m, nn = t.n;
    const bool diag = t.i0 == t.j0;
    const T* blk = Z + t.off;
    cd* s1 = slots + slot_base[blockIdx.x] * nrhs;
    cd* s2 = s1 + (int64_t)m * nrhs;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (int c0 = 0; c0 < nrhs; c0 += S) {
        const int cs = min(S, nrhs - c0);
        if (!cols_live(mk, c0, cs)) continue;
        __syncthreads();
        for (int e = tid; e < m * cs; e += NT) xi[e] = to_arith<A>(x[t.i0 + e % m + (int64_t)(c0 + e / m) * n]);
        for (int e = tid; e < nn * cs; e += NT) xj[e] = to_arith<A>(x[t.j0 + e % nn + (int64_t)(c0 + e / nn) * n]);
        __syncthreads();
        A cacc[2][S];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < S; ++c) cacc[q][c] = czero<A>();
        for (int a0 = wid; a0 < m; a0 += NW * RU) {
            A z[RU][2];
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int a = a0 + u * NW, b = lane + q * kWave;
                    z[u][q] = (a < m && b < nn) ? to_arith<A>(blk[(int64_t)a * nn + b]) : czero<A>();
                }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int a = a0 + u * NW;
                A racc[S];
#pragma unroll
                for (int c = 0; c < S; ++c) racc[c] = czero<A>();
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int b = lane + q * kWave;
                    if (b < nn && a < m)
#pragma unroll
                        for (int c = 0; c < S; ++c)
                            if (c < cs) {
                                racc[c] = cfma(z[u][q], xj[b + c * nn], racc[c]);
                                cacc[q][c] = cfma(z[u][q], xi[a + c * m], cacc[q][c]);
                            }
                }
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    if (c < cs) {
                        const A r = wave_sum(racc[c]);
                        if (lane == 0 && a < m) s1[a + (int64_t)(c0 + c) * m] = to_cd(r);
                    }
                }
            }
        }
        if (!diag) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int b = lane + q * kWave;
                if (b < nn)
#pragma unroll
                    for (int c = 0; c < S; ++c)
                        if (c < cs) colp[wid][b + c * nn] = cacc[q][c];
            }
            __syncthreads();
            for (int e = tid; e < nn * cs; e += NT) {
                A sum = colp[0][e];
#pragma unroll
                for (int w = 1; w < NW; ++w) sum = cadd(sum, colp[w][e]);
                s2[e % nn + (int64_t)(c0 + e / nn) * nn] = to_cd(sum);
            }
        }
    }
}

// ---------------------------------------------------------------- far matvec
// A far block (t, s) with U (m x r, column-major) and V (r x nn, row-major)
// adds slot_t = U (V x_s) and slot_s = V^T (U^T x_t).
//
// Blocks of at most 64 x 64 points and rank <= kFarWaveRank take one wave
// each: lane j holds row j of U and column j of V for every rank term, so
// each factor is read once; t1 = V x_s and t2 = U^T x_t are wave sums and
// both slots follow from the registers. S right-hand sides per pass.
template <int S, class T>
__device__ __forceinline__ void far_wave(const ColMask& mk, const AcaTask& g, int r, const T* U, cd* st, const cd* x,
                                         int64_t n, int nrhs) {
    using A = arith_t<T>;
    constexpr int RS = kFarWaveRank;
    const int lane = threadIdx.x % kWave;
    const int m = g.m, nn = g.n;
    cd* ss = st + (int64_t)m * nrhs;
    const T* V = U + (int64_t)m * r;
    A u[RS], v[RS];
#pragma unroll
    for (int l = 0; l < RS; ++l) {
        u[l] = (l < r && lane < m) ? to_arith<A>(U[lane + (int64_t)l * m]) : czero<A>();
        v[l] = (l < r && lane < nn) ? to_arith<A>(V[(int64_t)l * nn + lane]) : czero<A>();
    }
    for (int c0 = 0; c0 < nrhs; c0 += S) {
        const int cs = min(S, nrhs - c0);
        if (!cols_live(mk, c0, cs)) continue;
        A xs[S], xt[S], ot[S], os[S];
#pragma unroll
        for (int c = 0; c < S; ++c) {
            xs[c] = (c < cs && lane < nn) ? to_arith<A>(x[g.s0 + lane + (int64_t)(c0 + c) * n]) : czero<A>();
            xt[c] = (c < cs && lane < m) ? to_arith<A>(x[g.t0 + lane + (int64_t)(c0 + c) * n]) : czero<A>();
            ot[c] = czero<A>();
            os[c] = czero<A>();
        }
#pragma unroll
        for (int l = 0; l < RS; ++l) {
            if (l < r) {
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const A t1 = wave_sum(cmul(v[l], xs[c]));
                    const A t2 = wave_sum(cmul(u[l], xt[c]));
                    ot[c] = cfma(u[l], t1, ot[c]);
                    os[c] = cfma(v[l], t2, os[c]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < S; ++c) {
            if (c < cs) {
                if (lane < m) st[lane + (int64_t)(c0 + c) * m] = to_cd(ot[c]);
                if (lane < nn) ss[lane + (int64_t)(c0 + c) * nn] = to_cd(os[c]);
            }
        }
    }
}

// Wave tasks [0, ntasks) of the arrays passed, NW per workgroup.
template <int S, class T>
__global__ void __launch_bounds__(NT)
k_far_wave(ColMask mk, const AcaTask* __restrict__ geom, const int* __restrict__ rank, T* const* __restrict__ uv,
           const int64_t* __restrict__ slot_base, int64_t ntasks, const cd* __restrict__ x, int64_t n, int nrhs,
           cd* __restrict__ slots) {
    const int64_t task = (int64_t)blockIdx.x * NW + threadIdx.x / kWave;
    if (task >= ntasks) return;
    far_wave<S, T>(mk, geom[task], rank[task], uv[task], slots + slot_base[task] * nrhs, x, n, nrhs);
}

// One column, one workgroup: the larger factor is read once. With A the
// smaller side and B the larger (element (i, l) of U at U[i + l m], of V^T at
// V[i + l n]; xA, xB and outA, outB the matching segments of x and slots):
//   tA[l] = sum_j A(j, l) xA[j]                 (rows of A^T, RU per wave)
//   outB[i] = sum_l B(i, l) tA[l],  tB[l] = sum_i B(i, l) xB[i]
//                                               (B streamed once, by waves of
//                                                RB x 64 rows; per-wave partial
//                                                tB summed in wave order)
//   outA[j] = sum_l A(j, l) tB[l]               (one thread per row)
template <class T, int RU, int JU, int LG, class A = arith_t<T>>
__device__ __forceinline__ void far_wg_once(const AcaTask& g, int r, const T* U, const cd* x, cd* st, A* tA, A* tB,
                                            A (*tp)[kMaxRankCap]) {
    constexpr int RB = 4, LB = 2;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int m = g.m, nn = g.n;
    const T* V = U + (int64_t)m * r;
    const bool ubig = m >= nn;
    const T* Ab = ubig ? V : U;
    const T* Bb = ubig ? U : V;
    const int lenA = ubig ? nn : m, lenB = ubig ? m : nn;
    const cd* xA = x + (ubig ? g.s0 : g.t0);
    const cd* xB = x + (ubig ? g.t0 : g.s0);
    cd* outA = ubig ? st + m : st;
    cd* outB = ubig ? st : st + m;
    // tA: rows of A^T, JU column groups per step
    for (int l0 = wid; l0 < r; l0 += NW * RU) {
        A acc[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) acc[u] = czero<A>();
        for (int j0 = 0; j0 < lenA; j0 += JU * kWave) {
            A val[JU][RU], xv[JU];
#pragma unroll
            for (int jj = 0; jj < JU; ++jj) {
                const int j = j0 + jj * kWave + lane;
                xv[jj] = j < lenA ? to_arith<A>(xA[j]) : czero<A>();
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const int l = l0 + u * NW;
                    val[jj][u] = (l < r && j < lenA) ? to_arith<A>(Ab[(int64_t)l * lenA + j]) : czero<A>();
                }
            }
#pragma unroll
            for (int jj = 0; jj < JU; ++jj)
#pragma unroll
                for (int u = 0; u < RU; ++u) acc[u] = cfma(val[jj][u], xv[jj], acc[u]);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + u * NW;
            const A sum = wave_sum(acc[u]);
            if (lane == 0 && l < r) tA[l] = sum;
        }
    }
    for (int l = lane; l < r; l += kWave) tp[wid][l] = czero<A>();
    __syncthreads();
    // B once: its output rows and the per-wave partials of tB
    for (int i0 = wid * kWave * RB; i0 < lenB; i0 += NW * kWave * RB) {
        A xi[RB], o[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int i = i0 + k * kWave + lane;
            xi[k] = i < lenB ? to_arith<A>(xB[i]) : czero<A>();
            o[k] = czero<A>();
        }
        for (int l0 = 0; l0 < r; l0 += LB) {
            A bv[LB][RB];
#pragma unroll
            for (int u = 0; u < LB; ++u)
#pragma unroll
                for (int k = 0; k < RB; ++k) {
                    const int i = i0 + k * kWave + lane;
                    bv[u][k] = (l0 + u < r && i < lenB) ? to_arith<A>(Bb[i + (int64_t)(l0 + u) * lenB]) : czero<A>();
                }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                if (l0 + u < r) {
                    const A ta = tA[l0 + u];
                    A p = cmul(bv[u][0], xi[0]);
#pragma unroll
                    for (int k = 1; k < RB; ++k) p = cfma(bv[u][k], xi[k], p);
#pragma unroll
                    for (int k = 0; k < RB; ++k) o[k] = cfma(bv[u][k], ta, o[k]);
                    p = wave_sum(p);
                    if (lane == 0) tp[wid][l0 + u] = cadd(tp[wid][l0 + u], p);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int i = i0 + k * kWave + lane;
            if (i < lenB) outB[i] = to_cd(o[k]);
        }
    }
    __syncthreads();
    for (int l = tid; l < r + LG; l += NT) {
        A sum = czero<A>();
        if (l < r) {
            sum = tp[0][l];
#pragma unroll
            for (int w = 1; w < NW; ++w) sum = cadd(sum, tp[w][l]);
        }
        tB[l] = sum;   // zero padding past r for the grouped loads below
    }
    __syncthreads();
    // A's output rows, LG rank terms' loads issued together
    for (int j = tid; j < lenA; j += NT) {
        A acc = czero<A>();
        for (int l0 = 0; l0 < r; l0 += LG) {
            A av[LG];
#pragma unroll
            for (int u = 0; u < LG; ++u) av[u] = (l0 + u < r) ? to_arith<A>(Ab[j + (int64_t)(l0 + u) * lenA]) : czero<A>();
#pragma unroll
            for (int u = 0; u < LG; ++u) acc = cfma(av[u], tB[l0 + u], acc);
        }
        outA[j] = to_cd(acc);
    }
}

// The other blocks take one workgroup each: t1 and t2 (the 2r rows of V and
// of U^T, one wave per row, RU rows' loads issued together), then slot_t and
// slot_s (one thread per output row, LG rank terms' loads issued together).
// Single-column passes use far_wg_once instead.
// Workgroups [0, nwg) take tasks [0, nwg) (largest first); the rest take
// NW wave tasks each from nwg on. One launch covers every far block, so the
// small blocks fill the machine while the largest ones run.
template <int S, class T>
__global__ void __launch_bounds__(NT)
k_far_mv(ColMask mk, const AcaTask* __restrict__ geom, const int* __restrict__ rank, T* const* __restrict__ uv,
         const int64_t* __restrict__ slot_base, const cd* __restrict__ x, int64_t n, int nrhs,
         cd* __restrict__ slots) {
    using A = arith_t<T>;
    // one column: two column groups per step; sized for 5 waves per SIMD
    constexpr int RU = 4, JU = S == 1 ? 2 : 1, LG = 8;
    __shared__ A t12[2 * (kMaxRankCap + LG) * S];
    __shared__ A tpart[S == 1 ? NW : 1][kMaxRankCap];
    const AcaTask g = geom[blockIdx.x];
    const int m = g.m, nn = g.n, r = rank[blockIdx.x];
    if (r == 0) {
        cd* st = slots + slot_base[blockIdx.x] * nrhs;
        for (int64_t e = threadIdx.x; e < (int64_t)(m + nn) * nrhs; e += NT) st[e] = cmk(0.0, 0.0);
        return;
    }
    const T* U = uv[blockIdx.x];
    const T* V = U + (int64_t)m * r;
    cd* st = slots + slot_base[blockIdx.x] * nrhs;
    cd* ss = st + (int64_t)m * nrhs;
    if constexpr (S == 1) {   // nrhs is 1 here
        if (cols_live(mk, 0, 1)) far_wg_once<T, RU, JU, LG>(g, r, U, x, st, t12, t12 + kMaxRankCap + LG, tpart);
        return;
    }
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int rp = r + LG;   // t1 rows [0, r), padding, t2 rows from rp
    const int len_max = max(m, nn);
    for (int c0 = 0; c0 < nrhs; c0 += S) {
        const int cs = min(S, nrhs - c0);
        if (!cols_live(mk, c0, cs)) continue;
        __syncthreads();
        for (int l0 = wid; l0 < 2 * r; l0 += NW * RU) {
            A acc[RU][S];
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int c = 0; c < S; ++c) acc[u][c] = czero<A>();
            // JU column groups per step; x_s and x_t are read once per group
            // and shared by the rows (entries past a row's end are zero)
            for (int j0 = 0; j0 < len_max; j0 += JU * kWave) {
                A val[JU][RU], xsv[JU][S], xtv[JU][S];
#pragma unroll
                for (int jj = 0; jj < JU; ++jj) {
                    const int j = j0 + jj * kWave + lane;
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        xsv[jj][c] = (c < cs && j < nn) ? to_arith<A>(x[g.s0 + j + (int64_t)(c0 + c) * n]) : czero<A>();
                        xtv[jj][c] = (c < cs && j < m) ? to_arith<A>(x[g.t0 + j + (int64_t)(c0 + c) * n]) : czero<A>();
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const int l = l0 + u * NW;
                        const bool isv = l < r;
                        const int len = isv ? nn : m;
                        const T* row = isv ? V + (int64_t)l * nn : U + (int64_t)(l - r) * m;
                        val[jj][u] = (l < 2 * r && j < len) ? to_arith<A>(row[j]) : czero<A>();
                    }
                }
#pragma unroll
                for (int jj = 0; jj < JU; ++jj)
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const bool isv = l0 + u * NW < r;
#pragma unroll
                        for (int c = 0; c < S; ++c)
                            acc[u][c] = cfma(val[jj][u], isv ? xsv[jj][c] : xtv[jj][c], acc[u][c]);
                    }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int l = l0 + u * NW;
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    const A sum = wave_sum(acc[u][c]);
                    if (lane == 0 && l < 2 * r) t12[((l < r) ? l : rp + (l - r)) * S + c] = sum;
                }
            }
        }
        // zero padding so the grouped loads below read finite values
        if (tid < LG * S) {
            t12[r * S + tid] = czero<A>();
            t12[(rp + r) * S + tid] = czero<A>();
        }
        __syncthreads();
        for (int e = tid; e < m + nn; e += NT) {
            const bool top = e < m;
            const int idx = top ? e : e - m;
            const int ld = top ? m : nn;
            const T* base = (top ? U : V) + idx;
            const A* tv = t12 + (top ? 0 : rp) * S;
            A acc[S];
#pragma unroll
            for (int c = 0; c < S; ++c) acc[c] = czero<A>();
            for (int l0 = 0; l0 < r; l0 += LG) {
                A bv[LG];
#pragma unroll
                for (int u = 0; u < LG; ++u) bv[u] = (l0 + u < r) ? to_arith<A>(base[(int64_t)(l0 + u) * ld]) : czero<A>();
#pragma unroll
                for (int u = 0; u < LG; ++u)
#pragma unroll
                    for (int c = 0; c < S; ++c) acc[c] = cfma(bv[u], tv[(l0 + u) * S + c], acc[c]);
            }
            cd* out = top ? st : ss;
#pragma unroll
            for (int c = 0; c < S; ++c)
                if (c < cs) out[idx + (int64_t)(c0 + c) * ld] = to_cd(acc[c]);
        }
    }
}

// ---------------------------------------------------------------- gather
// y on leaf L = sum of the slots that cover it. The four waves of the
// workgroup take the leaf's gather entries in turn and their partial sums are
// added in wave order, so the result does not depend on timing. Each wave
// reads the descriptors of up to 64 of its entries at once (one per lane)
// and hands them to all lanes by lane reads, so the slot loads (GR in flight
// per lane) wait for one descriptor round trip per 64 entries, not per GR.
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ void __launch_bounds__(NT)
k_gather(ColMask mk, const int64_t* __restrict__ leaf_off, const int64_t* __restrict__ gptr,
         const GatherEnt* __restrict__ gent, const cd* __restrict__ slots, int64_t n, int nrhs, cd* __restrict__ y) {
    constexpr int GR = 8;
    __shared__ cd part[NW][kWave];
    const int64_t L = blockIdx.x;
    const int64_t i0 = leaf_off[L];
    const int b = (int)(leaf_off[L + 1] - i0);
    const int64_t e0 = gptr[L], e1 = gptr[L + 1];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    for (int base = 0; base < b * nrhs; base += kWave) {
        const int e = base + lane;
        const bool ok = e < b * nrhs;
        const int a = ok ? e % b : 0, c = ok ? e / b : 0;
        const bool live = ok && col_live(mk, c);
        cd acc = cmk(0.0, 0.0);
        // this wave's entries are e0 + wid + k NW, k = 0, 1, ...; chunks of 64
        for (int64_t q0 = e0 + wid; q0 < e1; q0 += (int64_t)NW * kWave) {
            const int64_t ql = q0 + (int64_t)lane * NW;
            GatherEnt gd{0, 0, 0};
            if (ql < e1) gd = gent[ql];
            const int cnt = (int)min<int64_t>(kWave, (e1 - q0 + NW - 1) / NW);
            for (int u0 = 0; u0 < cnt; u0 += GR) {
                cd v[GR];
#pragma unroll
                for (int u = 0; u < GR; ++u) {
                    const int src = min(u0 + u, cnt - 1);
                    const int64_t gb = readlane_i64(gd.base, src);
                    const int gl = __builtin_amdgcn_readlane(gd.len, src);
                    const int go = __builtin_amdgcn_readlane(gd.off, src);
                    v[u] = (live && u0 + u < cnt) ? slots[gb * nrhs + go + a + (int64_t)c * gl] : cmk(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < GR; ++u)
                    if (u0 + u < cnt) acc = cadd(acc, v[u]);
            }
        }
        part[wid][lane] = acc;
        __syncthreads();
        if (wid == 0 && live) {
            cd sum = part[0][lane];
#pragma unroll
            for (int w = 1; w < NW; ++w) sum = cadd(sum, part[w][lane]);
            y[i0 + a + (int64_t)c * n] = sum;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- GMRES pieces
int gmres_nchunk(int64_t n) {
    int64_t c = (n + NT - 1) / NT;
    if (c < 1) c = 1;
    if (c > 128) c = 128;
    return (int)c;
}

namespace {
__device__ __forceinline__ void chunk_range(int64_t n, int nchunk, int ch, int64_t& i0, int64_t& i1) {
    const int64_t len = (n + nchunk - 1) / nchunk;
    i0 = ch * len;
    i1 = min(n, i0 + len);
}

// Sum of the chunks' partials of column c, by the whole workgroup in a fixed order.
__device__ __forceinline__ double sum_chunks(const double* __restrict__ p, int nchunk, int nrhs, int c, double* red) {
    double s = 0.0;
    for (int q = threadIdx.x; q < nchunk; q += NT) s += p[(int64_t)q * nrhs + c];
    return wg_sum<NT>(s, red);
}
}  // namespace

// partial[(ch * nrhs + c) * nvec + l] = sum_{i in chunk} conj(V_l[i, c]) w[i, c].
// The vectors in groups of DG, one group per wave at a time (the waves work
// on different groups at once); a wave's lanes take the chunk's rows in
// turn, with a group's loads for two rows in flight together.
__global__ void __launch_bounds__(NT)
k_dots(const cd* __restrict__ V, int64_t ldv, int64_t vstride, int nvec, const cd* __restrict__ w, int64_t n,
       int nrhs, const ColState* __restrict__ st, cd* __restrict__ partial, int nchunk) {
    constexpr int DG = 8;
    const int ch = blockIdx.x, c = blockIdx.y;
    if (!st[c].active) return;
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int ngroups = (nvec + DG - 1) / DG;
    cd* pc = partial + ((int64_t)ch * nrhs + c) * nvec;
    for (int gi = wid; gi < ngroups; gi += NW) {
        const int l0 = gi * DG;
        cd acc[DG];
#pragma unroll
        for (int u = 0; u < DG; ++u) acc[u] = cmk(0.0, 0.0);
#pragma unroll 2
        for (int64_t i = i0 + lane; i < i1; i += kWave) {
            const cd wi = w[c * n + i];
            const cd* vb = V + c * ldv + i;
            cd vv[DG];
#pragma unroll
            for (int u = 0; u < DG; ++u) vv[u] = (l0 + u < nvec) ? vb[(int64_t)(l0 + u) * vstride] : cmk(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < DG; ++u) acc[u] = cfmac(vv[u], wi, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < DG; ++u) {
            const cd sum = wave_sum(acc[u]);
            if (lane == 0 && l0 + u < nvec) pc[l0 + u] = sum;
        }
    }
}

// h = sum over chunks of the partials; H_c(l, hcol) (+)= h_l; w -= V h;
// optionally the chunk's |w|^2 partial. H_c is (m + 1) x m column-major at
// H + c * ldh with ldh = (m + 1) m.
__global__ void __launch_bounds__(NT)
k_basis_update(const cd* __restrict__ V, int64_t ldv, int64_t vstride, int nvec, const cd* __restrict__ partial,
               int nchunk, cd* __restrict__ w, int64_t n, int nrhs, const ColState* __restrict__ st, cd* __restrict__ H,
               int64_t ldh, int mp1, int hcol, int accumulate_h, double* __restrict__ norm_partial) {
    constexpr int DG = 32;
    __shared__ cd h[kMaxRankCap + DG];
    __shared__ cd hp[NW][kWave];
    __shared__ double red[NW];
    const int ch = blockIdx.x, c = blockIdx.y;
    if (!st[c].active) return;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    for (int l0 = 0; l0 < nvec; l0 += kWave) {
        const int l = l0 + lane;
        cd s = cmk(0.0, 0.0);
        if (l < nvec) {
#pragma unroll 8
            for (int q = wid; q < nchunk; q += NW) s = cadd(s, partial[((int64_t)q * nrhs + c) * nvec + l]);
        }
        hp[wid][lane] = s;
        __syncthreads();
        if (threadIdx.x < kWave && l < nvec) {
            cd t = hp[0][lane];
#pragma unroll
            for (int q = 1; q < NW; ++q) t = cadd(t, hp[q][lane]);
            h[l] = t;
            if (ch == 0) {
                cd* hq = H + c * ldh + l + (int64_t)hcol * mp1;
                *hq = accumulate_h ? cadd(*hq, t) : t;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < DG) h[nvec + threadIdx.x] = cmk(0.0, 0.0);
    __syncthreads();
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    cd* wc = w + c * n;
    double ss = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
        cd v = wc[i];
        const cd* vb = V + c * ldv + i;
        for (int l0 = 0; l0 < nvec; l0 += DG) {
            cd vv[DG];
#pragma unroll
            for (int u = 0; u < DG; ++u) vv[u] = (l0 + u < nvec) ? vb[(int64_t)(l0 + u) * vstride] : cmk(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < DG; ++u) v = csub(v, cmul(vv[u], h[l0 + u]));
        }
        wc[i] = v;
        ss += cabs2(v);
    }
    if (norm_partial) {
        ss = wg_sum<NT>(ss, red);
        if (threadIdx.x == 0) norm_partial[(int64_t)ch * nrhs + c] = ss;
    }
}

namespace {
// Thread 0's part of k_givens_scale on the staged column Hc (j + 2 entries) and
// rotations cl / sl: earlier rotations, the new one (stored to cs / sn and
// cl / sl), the residual estimate and the stopping test.
__device__ void givens_column(cd* Hc, double* cl, cd* sl, int j, double hn, int m, ColState& s, cd* gc, double* cs,
                              cd* sn) {
    Hc[j + 1] = cmk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const cd a = Hc[i], b = Hc[i + 1];
        const cd t = cadd(cscale(a, cl[i]), cmul(sl[i], b));
        Hc[i + 1] = csub(cscale(b, cl[i]), cmul(cconj(sl[i]), a));
        Hc[i] = t;
    }
    const cd a = Hc[j];
    const double aa = sqrt(cabs2(a));
    double cc;
    cd ss;
    if (aa == 0.0) {
        cc = 0.0;
        ss = cmk(1.0, 0.0);
    } else {
        const double d = sqrt(aa * aa + hn * hn);
        cc = aa / d;
        ss = cscale(cmk(a.x / aa, a.y / aa), hn / d);   // (a/|a|) conj(b) / d with b = hn real
    }
    cs[j] = cc;
    sn[j] = ss;
    Hc[j] = cadd(cscale(a, cc), cscale(ss, hn));
    Hc[j + 1] = cmk(0.0, 0.0);
    const cd gj = gc[j];
    gc[j + 1] = cmul(cmk(-ss.x, ss.y), gj);   // -conj(s) g_j
    gc[j] = cscale(gj, cc);
    s.steps += 1;
    s.total += 1;
    bool stop = false;
    if (!s.fixed && sqrt(cabs2(gc[j + 1])) / s.bnorm <= s.tol) stop = true;
    if (s.total >= s.budget || hn == 0.0) stop = true;
    if (s.steps >= m) stop = true;
    if (stop) s.active = 0;
}
}  // namespace

// The end of one Arnoldi step, in one launch. Workgroup x = 0 of column
// c = y forms the Hessenberg column j: h_{j+1,j} = ||w||, the previous
// rotations, a new complex Givens rotation (real cosine), the residual
// estimate g and the column's stopping test. The other workgroups scale w
// into v_{j+1} by 1 / h_{j+1,j}; every workgroup sums the same norm partials
// in the same order, so all use the same h_{j+1,j}. A column that stops at
// this step may be scaled or not (its v_{j+1} is never read).
__global__ void __launch_bounds__(NT)
k_givens_scale(cd* __restrict__ H, int64_t ldh, int m, int j, double* __restrict__ csv, cd* __restrict__ snv,
               cd* __restrict__ g, const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st,
               int nrhs, const cd* __restrict__ w, cd* __restrict__ vnext, int64_t ldv, int64_t n) {
    __shared__ double red[NW];
    // the column and the earlier rotations, staged by the whole workgroup so
    // that the sequential rotations read LDS instead of dependent global loads
    __shared__ cd hcol[kMaxRankCap + 1], snl[kMaxRankCap];
    __shared__ double csl[kMaxRankCap];
    const int c = blockIdx.y;
    if (!st[c].active) return;
    if (blockIdx.x > 0) {
        const double hn = sqrt(sum_chunks(norm_partial, nchunk, nrhs, c, red));
        const double sc = hn > 0.0 ? 1.0 / hn : 0.0;
        const int64_t stride = (int64_t)(gridDim.x - 1) * NT;
        for (int64_t i = (blockIdx.x - 1) * (int64_t)NT + threadIdx.x; i < n; i += stride)
            vnext[c * ldv + i] = cscale(w[c * n + i], sc);
        return;
    }
    const int mp1 = m + 1;
    cd* Hg = H + c * ldh + (int64_t)j * mp1;
    double* cs = csv + (int64_t)c * m;
    cd* sn = snv + (int64_t)c * m;
    for (int i = threadIdx.x; i <= j; i += NT) hcol[i] = Hg[i];
    for (int i = threadIdx.x; i < j; i += NT) {
        csl[i] = cs[i];
        snl[i] = sn[i];
    }
    const double nn = sum_chunks(norm_partial, nchunk, nrhs, c, red);   // its barriers order the staging
    if (threadIdx.x == 0) {
        ColState s = st[c];
        const double hn = sqrt(nn);
        cd* gc = g + (int64_t)c * mp1;
        givens_column(hcol, csl, snl, j, hn, m, s, gc, cs, sn);
        st[c] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += NT) Hg[i] = hcol[i];
}

// Start of a restart cycle: beta = ||r||, V_0 = r / beta, g = (beta, 0, ...).
__global__ void __launch_bounds__(NT)
k_cycle_start(const cd* __restrict__ r, cd* __restrict__ V, int64_t ldv, cd* __restrict__ g, int m,
              const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st, int64_t n, int nrhs,
              int first) {
    __shared__ double red[NW];
    const int ch = blockIdx.x, c = blockIdx.y;
    const double beta = sqrt(sum_chunks(norm_partial, nchunk, nrhs, c, red));
    ColState s = st[c];
    if (first) {   // a column marked done beforehand stays done
        s.bnorm = beta;
        s.relres = beta > 0.0 ? 1.0 : 0.0;
        s.total = 0;
        s.done = (s.done || !(beta > 0.0)) ? 1 : 0;
    }
    const bool run = !s.done && beta > 0.0;
    if (ch == 0 && threadIdx.x == 0) {
        s.beta = beta;
        s.steps = 0;
        s.active = run ? 1 : 0;
        st[c] = s;
    }
    if (ch == 0)
        for (int i = threadIdx.x; i <= m; i += NT) g[(int64_t)c * (m + 1) + i] = cmk(i == 0 ? beta : 0.0, 0.0);
    if (!run) return;
    const double inv = 1.0 / beta;
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) V[c * ldv + i] = cscale(r[c * n + i], inv);
}

// Fresh column states: tolerance, step budget; a column is done from the
// start where the outer column (if given) is not active.
__global__ void k_col_init(ColState* __restrict__ st, const ColState* __restrict__ outer, int nrhs, double tol,
                           int budget) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    ColState s;
    s.bnorm = s.beta = s.relres = 0.0;
    s.tol = tol;
    s.active = s.steps = s.total = 0;
    s.done = (outer && !outer[c].active) ? 1 : 0;
    s.budget = budget;
    s.fixed = 0;
    s.pad0 = s.pad1 = 0;
    st[c] = s;
}

// Columns starting a solve inside a running multi-column solve (the listed
// slots): ||b|| from the chunk partials of b, and a fresh state, as the first
// cycle start of a solve sets it (relres 1, no steps; a zero b is done).
__global__ void __launch_bounds__(NT)
k_col_start(const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st, int nrhs,
            const int* __restrict__ cols, double tol, int budget, int fixed) {
    __shared__ double red[NW];
    const int c = cols[blockIdx.x];
    const double bn = sqrt(sum_chunks(norm_partial, nchunk, nrhs, c, red));
    if (threadIdx.x != 0) return;
    ColState s;
    s.bnorm = bn;
    s.beta = 0.0;
    s.relres = bn > 0.0 ? 1.0 : 0.0;
    s.tol = tol;
    s.active = s.steps = s.total = 0;
    s.done = bn > 0.0 ? 0 : 1;
    s.budget = budget;
    s.fixed = fixed;
    s.pad0 = s.pad1 = 0;
    st[c] = s;
}

// y = H^-1 g on the leading steps x steps triangle (back substitution).
__global__ void k_lsq(const cd* __restrict__ H, int64_t ldh, int m, const cd* __restrict__ g, cd* __restrict__ y,
                      const ColState* __restrict__ st, int nrhs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    const int k = st[c].steps;
    const int mp1 = m + 1;
    const cd* Hc = H + c * ldh;
    const cd* gc = g + (int64_t)c * mp1;
    cd* yc = y + (int64_t)c * m;
    for (int i = k - 1; i >= 0; --i) {
        cd s = gc[i];
        for (int l = i + 1; l < k; ++l) s = csub(s, cmul(Hc[i + (int64_t)l * mp1], yc[l]));
        yc[i] = cdiv(s, Hc[i + (int64_t)i * mp1]);
    }
}

// u = V[:, :steps] y (zero for columns with no step in this cycle).
__global__ void k_combine(const cd* __restrict__ V, int64_t ldv, int64_t vstride, const cd* __restrict__ y, int m,
                          cd* __restrict__ u, int64_t n, int nrhs, const ColState* __restrict__ st) {
    const int c = blockIdx.y;
    const int k = st[c].steps;
    const cd* yc = y + (int64_t)c * m;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cd s = cmk(0.0, 0.0);
        for (int l = 0; l < k; ++l) s = cfma(V[l * vstride + c * ldv + i], yc[l], s);
        u[c * n + i] = s;
    }
}

__global__ void k_axpy_x(cd* __restrict__ x, const cd* __restrict__ z, int64_t n, int nrhs,
                         const ColState* __restrict__ st) {
    const int c = blockIdx.y;
    if (st[c].steps == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[c * n + i] = cadd(x[c * n + i], z[c * n + i]);
}

// r = b - Z x and the chunks' |r|^2 partials.
__global__ void __launch_bounds__(NT)
k_residual(const cd* __restrict__ b, const cd* __restrict__ zx, cd* __restrict__ r, int64_t n, int nrhs,
           double* __restrict__ norm_partial, int nchunk) {
    __shared__ double red[NW];
    const int ch = blockIdx.x, c = blockIdx.y;
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    double ss = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
        const cd v = csub(b[c * n + i], zx[c * n + i]);
        r[c * n + i] = v;
        ss += cabs2(v);
    }
    ss = wg_sum<NT>(ss, red);
    if (threadIdx.x == 0) norm_partial[(int64_t)ch * nrhs + c] = ss;
}

__global__ void __launch_bounds__(NT)
k_col_norms(const cd* __restrict__ v, int64_t n, int nrhs, double* __restrict__ norm_partial, int nchunk) {
    __shared__ double red[NW];
    const int ch = blockIdx.x, c = blockIdx.y;
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    double ss = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) ss += cabs2(v[c * n + i]);
    ss = wg_sum<NT>(ss, red);
    if (threadIdx.x == 0) norm_partial[(int64_t)ch * nrhs + c] = ss;
}

// End of a cycle: true relative residual and the column's final stop test.
// One workgroup per column.
__global__ void __launch_bounds__(NT)
k_cycle_end(const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st, int nrhs) {
    __shared__ double red[NW];
    const int c = blockIdx.x;
    if (st[c].done) return;
    const double beta = sqrt(sum_chunks(norm_partial, nchunk, nrhs, c, red));
    if (threadIdx.x != 0) return;
    ColState s = st[c];
    s.relres = beta / s.bnorm;
    if (!isfinite(s.relres)) s.done = 1;
    if (!s.fixed && s.relres <= s.tol) s.done = 1;
    if (s.total >= s.budget || beta == 0.0) s.done = 1;
    s.active = 0;
    st[c] = s;
}

// ---------------------------------------------------------------- launchers
namespace {
inline unsigned grid1(int64_t n, int per = NT) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (unsigned)g;
}
}  // namespace

void launch_permute(const cd* src, cd* dst, const int64_t* perm, int64_t n, int64_t nrhs, bool to_tree, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(grid1(n * nrhs)), dim3(NT), 0, s, src, dst, perm, n, nrhs, (int)to_tree);
}

namespace {
template <class T>
void near_mv(const ColMask& mk, const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const T* Z, const cd* x,
             int64_t n, int nrhs, cd* slots, hipStream_t s) {
    if (ntasks == 0) return;
    if (nrhs == 1)
        hipLaunchKernelGGL((k_near_mv<1, T>), dim3((unsigned)ntasks), dim3(NT), 0, s, mk, tasks, slot_base, Z, x, n,
                           nrhs, slots);
    else
        hipLaunchKernelGGL((k_near_mv<SCH, T>), dim3((unsigned)ntasks), dim3(NT), 0, s, mk, tasks, slot_base, Z, x, n,
                           nrhs, slots);
}
template <class T>
void far_mv(const ColMask& mk, const AcaTask* geom, const int* rank, T* const* uv, const int64_t* slot_base,
            int64_t nwg, int64_t ntasks, const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    // the workgroup blocks, then the wave blocks: two kernels on one stream,
    // so each keeps its own register count (and occupancy)
    const int64_t nwv = ntasks - nwg;
    const unsigned gw = (unsigned)((nwv + NW - 1) / NW);
    if (nrhs == 1) {
        if (nwg > 0)
            hipLaunchKernelGGL((k_far_mv<1, T>), dim3((unsigned)nwg), dim3(NT), 0, s, mk, geom, rank, uv, slot_base, x,
                               n, nrhs, slots);
        if (nwv > 0)
            hipLaunchKernelGGL((k_far_wave<1, T>), dim3(gw), dim3(NT), 0, s, mk, geom + nwg, rank + nwg, uv + nwg,
                               slot_base + nwg, nwv, x, n, nrhs, slots);
    } else {
        if (nwg > 0)
            hipLaunchKernelGGL((k_far_mv<SCH, T>), dim3((unsigned)nwg), dim3(NT), 0, s, mk, geom, rank, uv, slot_base,
                               x, n, nrhs, slots);
        if (nwv > 0)
            hipLaunchKernelGGL((k_far_wave<SCH, T>), dim3(gw), dim3(NT), 0, s, mk, geom + nwg, rank + nwg, uv + nwg,
                               slot_base + nwg, nwv, x, n, nrhs, slots);
    }
}
}  // namespace

void launch_near_mv(const ColMask& mk, const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const cd* Z,
                    const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    near_mv(mk, tasks, slot_base, ntasks, Z, x, n, nrhs, slots, s);
}
void launch_near_mv(const ColMask& mk, const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const cf* Z,
                    const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    near_mv(mk, tasks, slot_base, ntasks, Z, x, n, nrhs, slots, s);
}
void launch_far_mv(const ColMask& mk, const AcaTask* geom, const int* rank, cd* const* uv, const int64_t* slot_base,
                   int64_t nwg, int64_t ntasks, const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    far_mv(mk, geom, rank, uv, slot_base, nwg, ntasks, x, n, nrhs, slots, s);
}
void launch_far_mv(const ColMask& mk, const AcaTask* geom, const int* rank, cf* const* uv, const int64_t* slot_base,
                   int64_t nwg, int64_t ntasks, const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    far_mv(mk, geom, rank, uv, slot_base, nwg, ntasks, x, n, nrhs, slots, s);
}

void launch_gather(const ColMask& mk, const int64_t* leaf_off, const int64_t* gptr, const GatherEnt* gent, int64_t nb,
                   const cd* slots, int64_t n, int nrhs, cd* y, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nb), dim3(NT), 0, s, mk, leaf_off, gptr, gent, slots, n, nrhs, y);
}

void launch_dots(const cd* V, int64_t ldv, int64_t vstride, int nvec, const cd* w, int64_t n, int nrhs,
                 const ColState* st, cd* partial, int nchunk, hipStream_t s) {
    hipLaunchKernelGGL(k_dots, dim3(nchunk, nrhs), dim3(NT), 0, s, V, ldv, vstride, nvec, w, n, nrhs, st, partial, nchunk);
}

void launch_basis_update(const cd* V, int64_t ldv, int64_t vstride, int nvec, const cd* partial, int nchunk, cd* w,
                         int64_t n, int nrhs, const ColState* st, cd* H, int64_t ldh, int mp1, int hcol,
                         bool accumulate_h, double* norm_partial, hipStream_t s) {
    hipLaunchKernelGGL(k_basis_update, dim3(nchunk, nrhs), dim3(NT), 0, s, V, ldv, vstride, nvec, partial, nchunk, w, n,
                       nrhs, st, H, ldh, mp1, hcol, (int)accumulate_h, norm_partial);
}

void launch_givens_scale(cd* H, int64_t ldh, int m, int j, double* cs, cd* sn, cd* g, const double* norm_partial,
                         int nchunk, ColState* st, int nrhs, const cd* w, cd* vnext, int64_t ldv, int64_t n,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_givens_scale, dim3(1 + grid1(n), nrhs), dim3(NT), 0, s, H, ldh, m, j, cs, sn, g, norm_partial,
                       nchunk, st, nrhs, w, vnext, ldv, n);
}

void launch_cycle_start(const cd* r, cd* V, int64_t ldv, cd* g, int m, const double* norm_partial, int nchunk,
                        ColState* st, int64_t n, int nrhs, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_start, dim3(nchunk, nrhs), dim3(NT), 0, s, r, V, ldv, g, m, norm_partial, nchunk, st, n,
                       nrhs, (int)first);
}

void launch_col_init(ColState* st, const ColState* outer, int nrhs, double tol, int budget, hipStream_t s) {
    hipLaunchKernelGGL(k_col_init, dim3((nrhs + 63) / 64), dim3(64), 0, s, st, outer, nrhs, tol, budget);
}

void launch_lsq(const cd* H, int64_t ldh, int m, const cd* g, cd* y, const ColState* st, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_lsq, dim3((nrhs + 63) / 64), dim3(64), 0, s, H, ldh, m, g, y, st, nrhs);
}

void launch_combine(const cd* V, int64_t ldv, int64_t vstride, const cd* y, int m, cd* u, int64_t n, int nrhs,
                    const ColState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(grid1(n), nrhs), dim3(NT), 0, s, V, ldv, vstride, y, m, u, n, nrhs, st);
}

void launch_axpy_x(cd* x, const cd* z, int64_t n, int nrhs, const ColState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_x, dim3(grid1(n), nrhs), dim3(NT), 0, s, x, z, n, nrhs, st);
}

void launch_residual(const cd* b, const cd* zx, cd* r, int64_t n, int nrhs, double* norm_partial, int nchunk,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(nchunk, nrhs), dim3(NT), 0, s, b, zx, r, n, nrhs, norm_partial, nchunk);
}

void launch_col_norms(const cd* v, int64_t n, int nrhs, double* norm_partial, int nchunk, hipStream_t s) {
    hipLaunchKernelGGL(k_col_norms, dim3(nchunk, nrhs), dim3(NT), 0, s, v, n, nrhs, norm_partial, nchunk);
}

void launch_col_start(const double* norm_partial, int nchunk, ColState* st, int nrhs, const int* cols, int ncols,
                      double tol, int budget, int fixed, hipStream_t s) {
    if (ncols > 0)
        hipLaunchKernelGGL(k_col_start, dim3(ncols), dim3(NT), 0, s, norm_partial, nchunk, st, nrhs, cols, tol, budget,
                           fixed);
}

void launch_cycle_end(const double* norm_partial, int nchunk, ColState* st, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_end, dim3(nrhs), dim3(NT), 0, s, norm_partial, nchunk, st, nrhs);
}

}  // namespace hs
