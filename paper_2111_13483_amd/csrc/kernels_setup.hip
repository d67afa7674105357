// gfx950 set-up kernels around the elimination:
//  * block copies (scatter of the near field into the working blocks W, D,
//    the dense part of the alpha store) and pointer-list copies;
//  * complex64 copies of stored blocks for the mixed-precision solve;
//  * a batched variable-size complex GEMM (64 x 64 output tiles, 4 x 4
//    complex register micro-tiles per thread, K staged through LDS), used for
//    the coupling products of the sweep plan.
#include "devcommon.h"
#include "kernels.h"

namespace hs {

namespace {
constexpr int NT = 256;
}

__global__ void __launch_bounds__(NT)
k_copy_blocks(const CopyTask* __restrict__ tasks, const cd* __restrict__ src, cd* __restrict__ dst) {
    const CopyTask t = tasks[blockIdx.x];
    const int rows = t.rows, cols = t.cols;
    const int64_t ld = t.dst_ld > 0 ? t.dst_ld : cols;
    cd* d = dst + t.dst_off;
    if (t.src_off < 0) {
        for (int e = threadIdx.x; e < rows * cols; e += NT) d[(e / cols) * ld + e % cols] = cmk(0.0, 0.0);
        return;
    }
    const cd* s = src + t.src_off;
    if (t.transpose) {
        for (int e = threadIdx.x; e < rows * cols; e += NT) {
            const int a = e / cols, b = e % cols;
            d[a * ld + b] = s[(int64_t)b * rows + a];
        }
    } else {
        for (int e = threadIdx.x; e < rows * cols; e += NT) d[(e / cols) * ld + e % cols] = s[e];
    }
}

__global__ void __launch_bounds__(NT) k_copy_ptrs(const PtrCopy* __restrict__ tasks, cd* __restrict__ dst) {
    const PtrCopy t = tasks[blockIdx.x];
    cd* d = dst + t.dst_off;
    for (int64_t e = threadIdx.x; e < t.count; e += NT) d[e] = t.src[e];
}

__global__ void __launch_bounds__(NT) k_copy_colmajor(const ColMajorCopy* __restrict__ tasks, cd* __restrict__ dst) {
    const ColMajorCopy t = tasks[blockIdx.x];
    cd* d = dst + t.dst_off;
    for (int e = threadIdx.x; e < t.rows * t.cols; e += NT) {
        const int i = e / t.cols, l = e % t.cols;
        d[e] = t.src[(int64_t)l * t.rows + i];
    }
}

// One workgroup per target block; element (i, j) of L^T T R is
// sum_p L[p][i] sum_q T[p][q] R[q][j], with identity factors skipped.
__global__ void __launch_bounds__(NT) k_core_expand(const CoreExpandTask* __restrict__ tasks, cd* __restrict__ base) {
    const CoreExpandTask t = tasks[blockIdx.x];
    const int ta = t.va ? t.ra : t.ba, tb = t.vb ? t.rb : t.bb;
    const cd* T = base + t.t_off;
    cd* D = base + t.dst_off;
    for (int e = threadIdx.x; e < t.ba * t.bb; e += NT) {
        const int i = e / t.bb, j = e % t.bb;
        cd acc = cmk(0.0, 0.0);
        for (int pp = 0; pp < ta; ++pp) {
            if (t.va == nullptr && pp != i) continue;
            cd row = cmk(0.0, 0.0);   // (T R)[pp][j]
            if (t.vb) {
                for (int q = 0; q < tb; ++q) row = cfma(T[(int64_t)pp * tb + q], t.vb[(int64_t)q * t.bb + j], row);
            } else {
                row = T[(int64_t)pp * tb + j];
            }
            acc = t.va ? cfma(t.va[(int64_t)pp * t.ba + i], row, acc) : row;
        }
        D[e] = cadd(D[e], acc);
    }
}

__global__ void __launch_bounds__(NT) k_to_c64(const PtrCopy* __restrict__ tasks, cf* __restrict__ dst) {
    const PtrCopy t = tasks[blockIdx.x];
    cf* d = dst + t.dst_off;
    for (int64_t e = threadIdx.x; e < t.count; e += NT) {
        const cd v = t.src[e];
        cf w;
        w.x = (float)v.x;
        w.y = (float)v.y;
        d[e] = w;
    }
}

// Complex GEMM of one task by one workgroup, 64 x 64 output tiles, 4 x 4
// complex register micro-tiles per thread, K staged through LDS:
// C (m x n) (+)= sign * op(A) B with op(A) = A (m x kk) or A^T (A kk x m).
template <bool TRANS_A>
__device__ __forceinline__ void gemm_task(const cd* __restrict__ A, const cd* __restrict__ B, cd* __restrict__ C, int m,
                                          int n, int kk, int accumulate, double sign) {
    constexpr int TM = 64, TN = 64, KC = 16;
    __shared__ cd As[KC][TM];
    __shared__ cd Bs[KC][TN];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    for (int m0 = 0; m0 < m; m0 += TM) {
        for (int n0 = 0; n0 < n; n0 += TN) {
            cd acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = cmk(0.0, 0.0);
            for (int k0 = 0; k0 < kk; k0 += KC) {
                __syncthreads();
                for (int e = tid; e < KC * TM; e += NT) {
                    const int l = e / TM, a = e % TM;
                    const int ga = m0 + a, gl = k0 + l;
                    cd v = cmk(0.0, 0.0);
                    if (ga < m && gl < kk) v = TRANS_A ? A[(int64_t)gl * m + ga] : A[(int64_t)ga * kk + gl];
                    As[l][a] = v;
                }
                for (int e = tid; e < KC * TN; e += NT) {
                    const int l = e / TN, c = e % TN;
                    const int gc = n0 + c, gl = k0 + l;
                    Bs[l][c] = (gc < n && gl < kk) ? B[(int64_t)gl * n + gc] : cmk(0.0, 0.0);
                }
                __syncthreads();
#pragma unroll 4
                for (int l = 0; l < KC; ++l) {
                    cd av[4], bv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) av[i] = As[l][ty * 4 + i];
#pragma unroll
                    for (int j = 0; j < 4; ++j) bv[j] = Bs[l][tx * 4 + j];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[i][j] = cfma(av[i], bv[j], acc[i][j]);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ga = m0 + ty * 4 + i;
                if (ga >= m) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int gc = n0 + tx * 4 + j;
                    if (gc >= n) continue;
                    cd v = cscale(acc[i][j], sign);
                    cd* dst = C + (int64_t)ga * n + gc;
                    *dst = accumulate ? cadd(*dst, v) : v;
                }
            }
        }
    }
}

// Batched GEMM, one task per workgroup, operands at offsets from shared bases.
template <bool TRANS_A>
__global__ void __launch_bounds__(NT)
k_gemm(const GemmTask* __restrict__ tasks, const cd* __restrict__ Ag, const cd* __restrict__ Bg, cd* __restrict__ Cg,
       int accumulate, double sign) {
    const GemmTask t = tasks[blockIdx.x];
    gemm_task<TRANS_A>(Ag + t.a_off, Bg + t.b_off, Cg + t.c_off, t.m, t.n, t.kk, accumulate, sign);
}

// C rows (64 per tile) = sum over k of A_row[k - k0] B[k][col]: one tile per
// workgroup, K staged through LDS, 4 x 4 complex micro-tiles per thread,
// ascending k from zero (rows add exact zeros outside their range).
__global__ void __launch_bounds__(NT)
k_chunk_gemm(const ChunkTile* __restrict__ tiles, const ChunkRow* __restrict__ rows, const cd* __restrict__ A,
             const cd* __restrict__ B, cd* __restrict__ C) {
    constexpr int TM = 64, TN = 64, KC = 16;
    __shared__ cd As[KC][TM];
    __shared__ cd Bs[KC][TN];
    __shared__ int64_t aoff[TM];
    __shared__ int rk0[TM], rkw[TM];
    const ChunkTile t = tiles[blockIdx.x];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    if (tid < TM) {
        if (tid < t.nrow) {
            const ChunkRow r = rows[t.row0 + tid];
            aoff[tid] = r.a_off;
            rk0[tid] = r.k0;
            rkw[tid] = r.kw;
        } else {
            aoff[tid] = 0;
            rk0[tid] = 0;
            rkw[tid] = 0;
        }
    }
    cd acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cmk(0.0, 0.0);
    // staging: thread tid serves row / column tid % 64, K rows tid / 64 + 4 u
    const int c = tid % TM, l0 = tid / TM;
    const int gc = t.col0 + c;
    for (int k0 = t.kmin; k0 < t.kmax; k0 += KC) {
        __syncthreads();
        cd av[KC / 4], bv[KC / 4];
#pragma unroll
        for (int u = 0; u < KC / 4; ++u) {
            const int k = k0 + l0 + 4 * u;
            const int lk = k - rk0[c];
            const bool oka = c < t.nrow && lk >= 0 && lk < rkw[c];
            av[u] = A[oka ? aoff[c] + lk : 0];
            const bool okb = k < t.kmax && gc < t.width;
            bv[u] = B[okb ? t.b_off + (int64_t)k * t.width + gc : 0];
            av[u] = oka ? av[u] : cmk(0.0, 0.0);
            bv[u] = okb ? bv[u] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < KC / 4; ++u) {
            As[l0 + 4 * u][c] = av[u];
            Bs[l0 + 4 * u][c] = bv[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int l = 0; l < KC; ++l) {
            cd a4[4], b4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a4[i] = As[l][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b4[j] = Bs[l][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = cfma(a4[i], b4[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = ty * 4 + i;
        if (rr >= t.nrow) continue;
        const int64_t co = rows[t.row0 + rr].c_off;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = t.col0 + tx * 4 + j;
            if (cc < t.width) C[co + cc] = acc[i][j];
        }
    }
}

void launch_chunk_gemm(const ChunkTile* tiles, int64_t ntiles, const ChunkRow* rows, const cd* A, const cd* B, cd* C,
                       hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_chunk_gemm, dim3((unsigned)ntiles), dim3(NT), 0, s, tiles, rows, A, B, C);
}

void launch_copy_blocks(const CopyTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_copy_blocks, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, src, dst);
}

void launch_copy_ptrs(const PtrCopy* tasks, int64_t ntasks, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_copy_ptrs, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, dst);
}

void launch_copy_colmajor(const ColMajorCopy* tasks, int64_t ntasks, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_copy_colmajor, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, dst);
}

void launch_core_expand(const CoreExpandTask* tasks, int64_t ntasks, cd* base, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_core_expand, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, base);
}

void launch_to_c64(const PtrCopy* tasks, int64_t ntasks, cf* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_to_c64, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, dst);
}

void launch_gemm(const GemmTask* tasks, int64_t ntasks, const cd* A, const cd* B, cd* C, bool transA, bool accumulate,
                 double sign, hipStream_t s) {
    if (ntasks == 0) return;
    if (transA)
        hipLaunchKernelGGL(k_gemm<true>, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, A, B, C, (int)accumulate, sign);
    else
        hipLaunchKernelGGL(k_gemm<false>, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, A, B, C, (int)accumulate, sign);
}

}  // namespace hs
