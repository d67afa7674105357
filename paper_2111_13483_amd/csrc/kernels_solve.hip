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
__global__ void __launch_bounds__(NT)
k_near_mv(const NearTask* __restrict__ tasks, const int64_t* __restrict__ slot_base, const cd* __restrict__ Z,
          const cd* __restrict__ x, int64_t n, int nrhs, cd* __restrict__ slots) {
    __shared__ cd xi[kMaxLeaf * SCH], xj[kMaxLeaf * SCH];
    __shared__ cd colp[NW][kMaxLeaf * SCH];
    const NearTask t = tasks[blockIdx.x];
    const int m = t.m, nn = t.n;
    const bool diag = t.i0 == t.j0;
    const cd* blk = Z + t.off;
    cd* s1 = slots + slot_base[blockIdx.x] * nrhs;
    cd* s2 = s1 + (int64_t)m * nrhs;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (int c0 = 0; c0 < nrhs; c0 += SCH) {
        const int cs = min(SCH, nrhs - c0);
        __syncthreads();
        for (int e = tid; e < m * cs; e += NT) xi[e] = x[t.i0 + e % m + (int64_t)(c0 + e / m) * n];
        for (int e = tid; e < nn * cs; e += NT) xj[e] = x[t.j0 + e % nn + (int64_t)(c0 + e / nn) * n];
        __syncthreads();
        cd cacc[2][SCH];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < SCH; ++c) cacc[q][c] = cmk(0.0, 0.0);
        for (int a = wid; a < m; a += NW) {
            cd racc[SCH];
#pragma unroll
            for (int c = 0; c < SCH; ++c) racc[c] = cmk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int b = lane + q * kWave;
                if (b < nn) {
                    const cd z = blk[(int64_t)a * nn + b];
#pragma unroll
                    for (int c = 0; c < SCH; ++c) {
                        if (c < cs) {
                            racc[c] = cfma(z, xj[b + c * nn], racc[c]);
                            cacc[q][c] = cfma(z, xi[a + c * m], cacc[q][c]);
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < SCH; ++c) {
                if (c < cs) {
                    cd r = wave_sum(racc[c]);
                    if (lane == 0) s1[a + (int64_t)(c0 + c) * m] = r;
                }
            }
        }
        if (!diag) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int b = lane + q * kWave;
                if (b < nn)
#pragma unroll
                    for (int c = 0; c < SCH; ++c)
                        if (c < cs) colp[wid][b + c * nn] = cacc[q][c];
            }
            __syncthreads();
            for (int e = tid; e < nn * cs; e += NT) {
                cd s = colp[0][e];
#pragma unroll
                for (int w = 1; w < NW; ++w) s = cadd(s, colp[w][e]);
                s2[e % nn + (int64_t)(c0 + e / nn) * nn] = s;
            }
        }
    }
}

// ---------------------------------------------------------------- far matvec
__global__ void __launch_bounds__(NT)
k_far_mv(const AcaTask* __restrict__ geom, const int* __restrict__ rank, cd* const* __restrict__ uv,
         const int64_t* __restrict__ slot_base, const cd* __restrict__ x, int64_t n, int nrhs, cd* __restrict__ slots) {
    __shared__ cd t1[kMaxRankCap * SCH], t2[kMaxRankCap * SCH];
    const AcaTask g = geom[blockIdx.x];
    const int m = g.m, nn = g.n, r = rank[blockIdx.x];
    const cd* U = uv[blockIdx.x];
    const cd* V = U + (int64_t)m * r;
    cd* st = slots + slot_base[blockIdx.x] * nrhs;
    cd* ss = st + (int64_t)m * nrhs;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const cd* xt = x + g.t0;
    const cd* xs = x + g.s0;
    for (int c0 = 0; c0 < nrhs; c0 += SCH) {
        const int cs = min(SCH, nrhs - c0);
        __syncthreads();
        for (int l = wid; l < r; l += NW) {
            cd a1[SCH], a2[SCH];
#pragma unroll
            for (int c = 0; c < SCH; ++c) { a1[c] = cmk(0.0, 0.0); a2[c] = cmk(0.0, 0.0); }
            const cd* vl = V + (int64_t)l * nn;
            const cd* ul = U + (int64_t)l * m;
            for (int j = lane; j < nn; j += kWave) {
                const cd v = vl[j];
#pragma unroll
                for (int c = 0; c < SCH; ++c)
                    if (c < cs) a1[c] = cfma(v, xs[j + (int64_t)(c0 + c) * n], a1[c]);
            }
            for (int i = lane; i < m; i += kWave) {
                const cd u = ul[i];
#pragma unroll
                for (int c = 0; c < SCH; ++c)
                    if (c < cs) a2[c] = cfma(u, xt[i + (int64_t)(c0 + c) * n], a2[c]);
            }
#pragma unroll
            for (int c = 0; c < SCH; ++c) {
                if (c < cs) {
                    cd s1 = wave_sum(a1[c]), s2v = wave_sum(a2[c]);
                    if (lane == 0) { t1[l * SCH + c] = s1; t2[l * SCH + c] = s2v; }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < m; i += NT) {
            cd acc[SCH];
#pragma unroll
            for (int c = 0; c < SCH; ++c) acc[c] = cmk(0.0, 0.0);
            for (int l = 0; l < r; ++l) {
                const cd u = U[(int64_t)l * m + i];
#pragma unroll
                for (int c = 0; c < SCH; ++c) acc[c] = cfma(u, t1[l * SCH + c], acc[c]);
            }
#pragma unroll
            for (int c = 0; c < SCH; ++c)
                if (c < cs) st[i + (int64_t)(c0 + c) * m] = acc[c];
        }
        for (int j = tid; j < nn; j += NT) {
            cd acc[SCH];
#pragma unroll
            for (int c = 0; c < SCH; ++c) acc[c] = cmk(0.0, 0.0);
            for (int l = 0; l < r; ++l) {
                const cd v = V[(int64_t)l * nn + j];
#pragma unroll
                for (int c = 0; c < SCH; ++c) acc[c] = cfma(v, t2[l * SCH + c], acc[c]);
            }
#pragma unroll
            for (int c = 0; c < SCH; ++c)
                if (c < cs) ss[j + (int64_t)(c0 + c) * nn] = acc[c];
        }
    }
}

// ---------------------------------------------------------------- gather
__global__ void __launch_bounds__(kWave)
k_gather(const int64_t* __restrict__ leaf_off, const int64_t* __restrict__ gptr, const GatherEnt* __restrict__ gent,
         const cd* __restrict__ slots, int64_t n, int nrhs, cd* __restrict__ y) {
    const int64_t L = blockIdx.x;
    const int64_t i0 = leaf_off[L];
    const int b = (int)(leaf_off[L + 1] - i0);
    const int64_t e0 = gptr[L], e1 = gptr[L + 1];
    for (int e = threadIdx.x; e < b * nrhs; e += kWave) {
        const int a = e % b, c = e / b;
        cd acc = cmk(0.0, 0.0);
        for (int64_t q = e0; q < e1; ++q) {
            const GatherEnt g = gent[q];
            acc = cadd(acc, slots[g.base * nrhs + g.off + a + (int64_t)c * g.len]);
        }
        y[i0 + a + (int64_t)c * n] = acc;
    }
}

// ---------------------------------------------------------------- GMRES pieces
int gmres_nchunk(int64_t n) {
    int64_t c = (n + 4095) / 4096;
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
}  // namespace

// partial[(ch * nrhs + c) * nvec + l] = sum_{i in chunk} conj(V_l[i, c]) w[i, c]
__global__ void __launch_bounds__(NT)
k_dots(const cd* __restrict__ V, int64_t ldv, int64_t vstride, int nvec, const cd* __restrict__ w, int64_t n,
       int nrhs, const ColState* __restrict__ st, cd* __restrict__ partial, int nchunk) {
    const int ch = blockIdx.x, c = blockIdx.y;
    if (!st[c].active) return;
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const cd* wc = w + c * n;
    for (int l = wid; l < nvec; l += NW) {
        const cd* vl = V + l * vstride + c * ldv;
        cd s = cmk(0.0, 0.0);
        for (int64_t i = i0 + lane; i < i1; i += kWave) s = cfmac(vl[i], wc[i], s);
        s = wave_sum(s);
        if (lane == 0) partial[((int64_t)ch * nrhs + c) * nvec + l] = s;
    }
}

// h = sum over chunks of the partials; H_c(l, hcol) (+)= h_l; w -= V h;
// optionally the chunk's |w|^2 partial. H_c is (m + 1) x m column-major at
// H + c * ldh with ldh = (m + 1) m.
__global__ void __launch_bounds__(NT)
k_basis_update(const cd* __restrict__ V, int64_t ldv, int64_t vstride, int nvec, const cd* __restrict__ partial,
               int nchunk, cd* __restrict__ w, int64_t n, int nrhs, const ColState* __restrict__ st, cd* __restrict__ H,
               int64_t ldh, int mp1, int hcol, int accumulate_h, double* __restrict__ norm_partial) {
    __shared__ cd h[kMaxRankCap + 1];
    __shared__ double red[NW];
    const int ch = blockIdx.x, c = blockIdx.y;
    if (!st[c].active) return;
    for (int l = threadIdx.x; l < nvec; l += NT) {
        cd s = cmk(0.0, 0.0);
        for (int q = 0; q < nchunk; ++q) s = cadd(s, partial[((int64_t)q * nrhs + c) * nvec + l]);
        h[l] = s;
        if (ch == 0) {
            cd* hp = H + c * ldh + l + (int64_t)hcol * mp1;
            *hp = accumulate_h ? cadd(*hp, s) : s;
        }
    }
    __syncthreads();
    int64_t i0, i1;
    chunk_range(n, nchunk, ch, i0, i1);
    cd* wc = w + c * n;
    double ss = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
        cd v = wc[i];
        for (int l = 0; l < nvec; ++l) v = csub(v, cmul(V[l * vstride + c * ldv + i], h[l]));
        wc[i] = v;
        ss += cabs2(v);
    }
    if (norm_partial) {
        ss = wg_sum<NT>(ss, red);
        if (threadIdx.x == 0) norm_partial[(int64_t)ch * nrhs + c] = ss;
    }
}

// One Arnoldi step's Hessenberg column j: h_{j+1,j} = ||w||, previous
// rotations, a new complex Givens rotation (real cosine), the residual
// estimate g and the column's stopping test. One thread per column.
__global__ void k_givens(cd* __restrict__ H, int64_t ldh, int m, int j, double* __restrict__ csv, cd* __restrict__ snv,
                         cd* __restrict__ g, const double* __restrict__ norm_partial, int nchunk,
                         ColState* __restrict__ st, int nrhs, double* __restrict__ inv_hn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    ColState s = st[c];
    if (!s.active) return;
    const int mp1 = m + 1;
    double nn = 0.0;
    for (int q = 0; q < nchunk; ++q) nn += norm_partial[(int64_t)q * nrhs + c];
    const double hn = sqrt(nn);
    cd* Hc = H + c * ldh + (int64_t)j * mp1;
    double* cs = csv + (int64_t)c * m;
    cd* sn = snv + (int64_t)c * m;
    cd* gc = g + (int64_t)c * mp1;
    Hc[j + 1] = cmk(hn, 0.0);
    for (int i = 0; i < j; ++i) {
        const cd a = Hc[i], b = Hc[i + 1];
        const cd t = cadd(cscale(a, cs[i]), cmul(sn[i], b));
        Hc[i + 1] = csub(cscale(b, cs[i]), cmul(cconj(sn[i]), a));
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
    inv_hn[c] = hn > 0.0 ? 1.0 / hn : 0.0;
    bool stop = false;
    if (!s.fixed && sqrt(cabs2(gc[j + 1])) / s.bnorm <= s.tol) stop = true;
    if (s.total >= s.budget || hn == 0.0) stop = true;
    if (s.steps >= m) stop = true;
    if (stop) s.active = 0;
    st[c] = s;
}

__global__ void k_scale_next(const cd* __restrict__ w, cd* __restrict__ vnext, int64_t ldv, int64_t n, int nrhs,
                             const ColState* __restrict__ st, const double* __restrict__ inv_hn) {
    const int c = blockIdx.y;
    if (!st[c].active) return;
    const double s = inv_hn[c];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        vnext[c * ldv + i] = cscale(w[c * n + i], s);
}

// Start of a restart cycle: beta = ||r||, V_0 = r / beta, g = (beta, 0, ...).
__global__ void __launch_bounds__(NT)
k_cycle_start(const cd* __restrict__ r, cd* __restrict__ V, int64_t ldv, cd* __restrict__ g, int m,
              const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st, int64_t n, int nrhs,
              int first) {
    const int ch = blockIdx.x, c = blockIdx.y;
    double nn = 0.0;
    for (int q = 0; q < nchunk; ++q) nn += norm_partial[(int64_t)q * nrhs + c];
    const double beta = sqrt(nn);
    ColState s = st[c];
    if (first) {
        s.bnorm = beta;
        s.relres = beta > 0.0 ? 1.0 : 0.0;
        s.total = 0;
        s.done = beta > 0.0 ? 0 : 1;
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
__global__ void k_cycle_end(const double* __restrict__ norm_partial, int nchunk, ColState* __restrict__ st, int nrhs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    ColState s = st[c];
    if (s.done) return;
    double nn = 0.0;
    for (int q = 0; q < nchunk; ++q) nn += norm_partial[(int64_t)q * nrhs + c];
    const double beta = sqrt(nn);
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

void launch_near_mv(const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const cd* Z, const cd* x, int64_t n,
                    int nrhs, cd* slots, hipStream_t s) {
    if (ntasks > 0)
        hipLaunchKernelGGL(k_near_mv, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, slot_base, Z, x, n, nrhs, slots);
}

void launch_far_mv(const AcaTask* geom, const int* rank, cd* const* uv, const int64_t* slot_base, int64_t ntasks,
                   const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s) {
    if (ntasks > 0)
        hipLaunchKernelGGL(k_far_mv, dim3((unsigned)ntasks), dim3(NT), 0, s, geom, rank, uv, slot_base, x, n, nrhs, slots);
}

void launch_gather(const int64_t* leaf_off, const int64_t* gptr, const GatherEnt* gent, int64_t nb, const cd* slots,
                   int64_t n, int nrhs, cd* y, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nb), dim3(kWave), 0, s, leaf_off, gptr, gent, slots, n, nrhs, y);
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

void launch_givens(cd* H, int64_t ldh, int m, int j, double* cs, cd* sn, cd* g, const double* norm_partial, int nchunk,
                   ColState* st, int nrhs, double* inv_hn, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, dim3((nrhs + 63) / 64), dim3(64), 0, s, H, ldh, m, j, cs, sn, g, norm_partial, nchunk,
                       st, nrhs, inv_hn);
}

void launch_scale_next(const cd* w, cd* vnext, int64_t ldv, int64_t n, int nrhs, const ColState* st,
                       const double* inv_hn, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_next, dim3(grid1(n), nrhs), dim3(NT), 0, s, w, vnext, ldv, n, nrhs, st, inv_hn);
}

void launch_cycle_start(const cd* r, cd* V, int64_t ldv, cd* g, int m, const double* norm_partial, int nchunk,
                        ColState* st, int64_t n, int nrhs, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_start, dim3(nchunk, nrhs), dim3(NT), 0, s, r, V, ldv, g, m, norm_partial, nchunk, st, n,
                       nrhs, (int)first);
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

void launch_cycle_end(const double* norm_partial, int nchunk, ColState* st, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_cycle_end, dim3((nrhs + 63) / 64), dim3(64), 0, s, norm_partial, nchunk, st, nrhs);
}

}  // namespace hs
