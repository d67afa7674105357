// gfx950 kernels of the H-matrix build and of every low-rank compression:
//  * near-field assembly of the scalar Helmholtz kernel (Eq. 5-7 kernel,
//    point collocation), one workgroup per stored near block;
//  * partial-pivoting ACA (Eq. 9-10), one workgroup per block, rows and
//    columns generated on the fly from the points (far field) or read from
//    a stored dense block (fill-in blocks of the scaling coefficients,
//    Sec. 3.4);
//  * re-compression (the text after Eq. 10): in-place QR of U and V^T by
//    classical Gram-Schmidt applied twice, one-sided complex Jacobi SVD of
//    the r x r core, truncation at the same relative Frobenius tolerance,
//    and the final factors U' = Q_U W S, V' = X^H Q_V^T.
#include "devcommon.h"
#include "kernels.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;
// Re-compression: one workgroup per block.
constexpr int NTR = 256;
// a factor with len * r <= kRcLds elements is factored in LDS, and the core
// with its rotations (2 r^2 <= kRcLds) rotated there; small enough (8 KB)
// that the kernel's occupancy stays bound by its registers
constexpr int kRcLds = 512;
// Blocks of rank above kRcWideRank: 1024 threads, and cores up to rank 45
// (2 r^2 <= 4096) rotated in LDS.
constexpr int NTW = 1024;
constexpr int kRcLdsWide = 4096;
// loads in flight per lane in the QR of the factors (registers: 1024-thread
// workgroups may take 128 VGPRs, the 256-thread ones share CUs with many)
constexpr int kQbWide = 8;
constexpr int kQbRest = 4;
// Lists of small blocks (kRcSmall): one wave each, factors of up to 64 x 8
// and cores up to rank 16 worked on in its 8 KB of LDS; ranks of at most
// kRcSmallLen (about 10 KB of LDS in all, 16 workgroups per CU).
constexpr int kRcLdsSmall = 512;
constexpr int kQbSmall = 2;
constexpr double kPi = 3.141592653589793238462643383279502884;

// exp(-j k r) / (4 pi r) with the products and sums rounded as written.
__device__ __forceinline__ cd green(const double* a, const double* b, double k) {
#pragma clang fp contract(off)
    double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double kr = k * r;
    double s, c;
    sincos(kr, &s, &c);
    double den = (4.0 * kPi) * r;
    return cmk(c / den, -s / den);
}

}  // namespace

__global__ void __launch_bounds__(NT)
k_near_assemble(const NearTask* __restrict__ tasks, const double* __restrict__ pts, double k, double h,
                cd* __restrict__ out, int* err) {
    const NearTask t = tasks[blockIdx.x];
    const int m = t.m, n = t.n;
    cd* blk = out + t.off;
    const bool same = t.i0 == t.j0;
    cd self;
    {
#pragma clang fp contract(off)
        double den = 2.0 * kPi * h;
        self = cmk(1.0 / den, -(k * h / 2.0) / den);
    }
    for (int e = threadIdx.x; e < m * n; e += NT) {
        const int a = e / n, b = e % n;
        if (same && a == b) {
            blk[e] = self;
            continue;
        }
        const double* pa = pts + 3 * (int64_t)(t.i0 + a);
        const double* pb = pts + 3 * (int64_t)(t.j0 + b);
        if (pa[0] == pb[0] && pa[1] == pb[1] && pa[2] == pb[2]) {
            raise_err(err, kErrCoincident);
            blk[e] = cmk(0.0, 0.0);
            continue;
        }
        // rows are observers: G(p_a, p_b); r is symmetric in its arguments
        blk[e] = green(pb, pa, k);
    }
}

namespace {

template <bool DENSE>
__device__ __forceinline__ cd src_val(const AcaTask& t, const double* pts, double k, const cd* dense, int i, int j) {
    if constexpr (DENSE) {
        return dense[t.src_off + (int64_t)i * t.n + j];
    } else {
        return green(pts + 3 * (int64_t)(t.s0 + j), pts + 3 * (int64_t)(t.t0 + i), k);
    }
}

}  // namespace

// Partial-pivoting ACA of one block per workgroup. U (m x cap, column-major)
// and V (cap x n, row-major) live in the task's scratch region; flags holds
// m + n "used" bytes.
template <bool DENSE>
__global__ void __launch_bounds__(NT)
k_aca(const AcaTask* __restrict__ tasks, const int* __restrict__ order, const double* __restrict__ pts, double k,
      const cd* __restrict__ dense, cd* __restrict__ scratch, uint8_t* __restrict__ flags, double eps,
      int* __restrict__ rank_out, int* __restrict__ piv_log, int piv_stride, int* err) {
    __shared__ double redv[NW];
    __shared__ int redi[NW];
    __shared__ double cross_part[NW];
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;   // the largest blocks first
    const AcaTask t = tasks[bi];
    const int m = t.m, n = t.n, cap = t.cap;
    cd* U = scratch + t.u_off;
    cd* V = scratch + t.v_off;
    uint8_t* rused = flags + t.flag_off;
    uint8_t* cused = rused + m;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (int x = tid; x < m + n; x += NT) rused[x] = 0;
    __syncthreads();
    const int rmax = min(min(m, n), cap);
    int rank = 0;
    double norm2 = 0.0;
    int i = 0;
    bool capped = false;
    while (rank < rmax) {
        // residual row i -> V[rank, :], and its largest entry over unused columns
        cd* vrow = V + (int64_t)rank * n;
        ArgMax am{-1.0, 0x7fffffff};
        for (int j = tid; j < n; j += NT) {
            cd v = src_val<DENSE>(t, pts, k, dense, i, j);
            for (int l = 0; l < rank; ++l) v = csub(v, cmul(U[(int64_t)l * m + i], V[(int64_t)l * n + j]));
            vrow[j] = v;
            if (!cused[j]) am = amax_pick(am, ArgMax{cabs2_exact(v), j});
        }
        am = wg_argmax<NT>(am, redv, redi);
        if (tid == 0) rused[i] = 1;
        __syncthreads();
        if (!(am.v > 0.0)) {
            // zero residual row: try the lowest unused row
            ArgMax f{-1.0, 0x7fffffff};
            for (int x = tid; x < m; x += NT)
                if (!rused[x]) f = amax_pick(f, ArgMax{(double)(m - x), x});
            f = wg_argmax<NT>(f, redv, redi);
            if (f.v < 0.0) break;
            i = f.i;
            continue;
        }
        const int js = am.i;
        const cd piv = vrow[js];
        __syncthreads();
        for (int j = tid; j < n; j += NT) vrow[j] = cdiv(vrow[j], piv);
        // residual column js -> U[:, rank]
        cd* ucol = U + (int64_t)rank * m;
        for (int x = tid; x < m; x += NT) {
            cd u = src_val<DENSE>(t, pts, k, dense, x, js);
            for (int l = 0; l < rank; ++l) u = csub(u, cmul(V[(int64_t)l * n + js], U[(int64_t)l * m + x]));
            ucol[x] = u;
        }
        __syncthreads();
        if (tid == 0) cused[js] = 1;
        double pu = 0.0, pv = 0.0;
        for (int x = tid; x < m; x += NT) pu += cabs2(ucol[x]);
        for (int x = tid; x < n; x += NT) pv += cabs2(vrow[x]);
        const double nu2 = wg_sum<NT>(pu, redv);
        const double nv2 = wg_sum<NT>(pv, redv);
        // cross terms 2 Re((u_l^H u)(v_l^H v)), one previous term per wave at a time
        double cr = 0.0;
        for (int l = wid; l < rank; l += NW) {
            cd du = cmk(0.0, 0.0), dv = cmk(0.0, 0.0);
            const cd* ul = U + (int64_t)l * m;
            const cd* vl = V + (int64_t)l * n;
            for (int x = lane; x < m; x += kWave) du = cfmac(ul[x], ucol[x], du);
            for (int x = lane; x < n; x += kWave) dv = cfmac(vl[x], vrow[x], dv);
            du = wave_sum(du);
            dv = wave_sum(dv);
            cr += du.x * dv.x - du.y * dv.y;
        }
        if (lane == 0) cross_part[wid] = cr;
        __syncthreads();
        double cross = 0.0;
        for (int w = 0; w < NW; ++w) cross += cross_part[w];
        norm2 += nu2 * nv2 + 2.0 * cross;
        if (tid == 0 && piv_log) {
            piv_log[(int64_t)bi * piv_stride + 2 * rank] = i;
            piv_log[(int64_t)bi * piv_stride + 2 * rank + 1] = js;
        }
        ++rank;
        if (sqrt(nu2 * nv2) <= eps * sqrt(fmax(norm2, 0.0))) break;
        if (rank >= rmax) {
            if (rmax < min(m, n)) capped = true;
            break;
        }
        // next row: largest |u| over unused rows
        ArgMax nx{-1.0, 0x7fffffff};
        for (int x = tid; x < m; x += NT)
            if (!rused[x]) nx = amax_pick(nx, ArgMax{cabs2_exact(ucol[x]), x});
        nx = wg_argmax<NT>(nx, redv, redi);
        if (nx.i == 0x7fffffff) break;
        i = nx.i;
    }
    if (tid == 0) {
        rank_out[bi] = rank;
        if (capped) raise_err(err, kErrRankCap);
    }
}

namespace {

// In-place QR of the r columns (each of length len, stride len) of A by
// classical Gram-Schmidt applied twice; R (r x r, column-major) receives the
// triangular factor. hbuf: LDS of >= r entries. The factors of the large
// blocks stay in global memory, so the dot products and the column update
// are unrolled QB times to keep QB loads per lane in flight (a column of
// 2,000 points is then 32 / QB rounds of load latency per lane).
template <int NTQ, int QB>
__device__ void cgs2_qr(cd* A, int len, int r, cd* R, cd* hbuf, double* red) {
    constexpr int NWQ = NTQ / kWave;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    for (int c = 0; c < r; ++c) {
        cd* ac = A + (int64_t)c * len;
        for (int pass = 0; pass < 2; ++pass) {
            for (int l = wid; l < c; l += NWQ) {
                const cd* al = A + (int64_t)l * len;
                cd d = cmk(0.0, 0.0);
#pragma unroll QB
                for (int x = lane; x < len; x += kWave) d = cfmac(al[x], ac[x], d);
                d = wave_sum(d);
                if (lane == 0) hbuf[l] = d;
            }
            __syncthreads();
            for (int x = tid; x < len; x += NTQ) {
                cd v = ac[x];
#pragma unroll QB
                for (int l = 0; l < c; ++l) v = csub(v, cmul(A[(int64_t)l * len + x], hbuf[l]));
                ac[x] = v;
            }
            for (int l = tid; l < c; l += NTQ) {
                cd prev = pass == 0 ? cmk(0.0, 0.0) : R[l + (int64_t)c * r];
                R[l + (int64_t)c * r] = cadd(prev, hbuf[l]);
            }
            __syncthreads();
        }
        double p = 0.0;
        for (int x = tid; x < len; x += NTQ) p += cabs2(ac[x]);
        const double nrm = sqrt(wg_sum<NTQ>(p, red));
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int x = tid; x < len; x += NTQ) ac[x] = cscale(ac[x], inv);
        if (tid == 0) R[c + (int64_t)c * r] = cmk(nrm, 0.0);
        for (int l = c + 1 + tid; l < r; l += NTQ) R[l + (int64_t)c * r] = cmk(0.0, 0.0);
        __syncthreads();
    }
}

// Sum over a row of 16 lanes, the same bits in every lane of the row: each
// DPP step adds the value of a partner lane whose group holds the same
// operands (quad_perm [1,0,3,2] and [2,3,0,1], then row_half_mirror pairing
// the two quads of each half, then row_mirror pairing the halves), so the
// lanes' sums differ only in operand order. The moves stay within the row,
// so only the row has to be active.
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return v;
}
__device__ __forceinline__ cd row_sum(cd v) { return cmk(row_sum(v.x), row_sum(v.y)); }

constexpr int kJr = 16;   // lanes per Jacobi pair: one DPP row

// One-sided Jacobi on the columns of M (r x r, column-major), accumulating
// the right rotations in X (starts as I). Round-robin pairs, one pair per
// row of 16 lanes at a time (a round's pairs are disjoint, so up to
// NTQ / 16 of them run at once; each lane takes every 16th entry).
template <int NTQ>
__device__ void jacobi_svd(cd* M, cd* X, int r, int* rot_flag) {
    constexpr int NG = NTQ / kJr;
    const int tid = threadIdx.x, gl = tid % kJr, grp = tid / kJr;
    const int np = (r + 1) & ~1;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) *rot_flag = 0;
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            for (int pk = grp; pk < np / 2; pk += NG) {
                int p, q;
                if (pk == 0) { p = round; q = np - 1; }
                else { p = (round + pk) % (np - 1); q = (round - pk + np - 1) % (np - 1); }
                if (p > q) { int tt = p; p = q; q = tt; }
                if (q >= r) continue;
                cd* mp = M + (int64_t)p * r;
                cd* mq = M + (int64_t)q * r;
                double a = 0.0, b = 0.0;
                cd c = cmk(0.0, 0.0);
                for (int x = gl; x < r; x += kJr) {
                    a += cabs2(mp[x]);
                    b += cabs2(mq[x]);
                    c = cfmac(mp[x], mq[x], c);
                }
                a = row_sum(a);
                b = row_sum(b);
                c = row_sum(c);
                const double ac = sqrt(cabs2(c));
                if (!(ac > 1e-15 * sqrt(a * b)) || ac == 0.0) continue;
                const double zeta = (b - a) / (2.0 * ac);
                const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
                const cd ph = cmk(c.x / ac, -c.y / ac);   // e^{-i phi}
                for (int x = gl; x < r; x += kJr) {
                    cd u = mp[x], w = cmul(ph, mq[x]);
                    mp[x] = cmk(cs * u.x - sn * w.x, cs * u.y - sn * w.y);
                    mq[x] = cmk(sn * u.x + cs * w.x, sn * u.y + cs * w.y);
                }
                cd* xp = X + (int64_t)p * r;
                cd* xq = X + (int64_t)q * r;
                for (int x = gl; x < r; x += kJr) {
                    cd u = xp[x], w = cmul(ph, xq[x]);
                    xp[x] = cmk(cs * u.x - sn * w.x, cs * u.y - sn * w.y);
                    xq[x] = cmk(sn * u.x + cs * w.x, sn * u.y + cs * w.y);
                }
                if (gl == 0) *rot_flag = 1;
            }
            __syncthreads();
        }
        const int any = *rot_flag;
        __syncthreads();
        if (!any) break;
    }
}

}  // namespace

// Re-compression, phase A: QR of U and V^T in place, core M = R_U R_V^T,
// Jacobi SVD, singular values sorted (descending, ties by index) and the
// truncated rank. Workgroup w takes block order[w] (the host lists the
// costliest blocks first, so the longest ones do not trail the launch; null:
// block w).
template <int NTQ, int LDSC, int QB, int RMX = kMaxRankCap>
__global__ void __launch_bounds__(NTQ)
k_recompress_a(const AcaTask* __restrict__ tasks, const int* __restrict__ order, cd* __restrict__ scratch,
               const int* __restrict__ rank_in, cd* __restrict__ ws, const int64_t* __restrict__ ws_off, double eps,
               int* __restrict__ rank_out) {
    __shared__ cd hbuf[RMX];
    __shared__ double red[NTQ / kWave];
    __shared__ int rot_flag;
    __shared__ double sig[RMX];
    __shared__ int srt[RMX];
    __shared__ cd lbuf[LDSC];
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const AcaTask t = tasks[bi];
    const int r = rank_in[bi];
    const int tid = threadIdx.x;
    if (r == 0) {
        if (tid == 0) rank_out[bi] = 0;
        return;
    }
    cd* U = scratch + t.u_off;
    cd* V = scratch + t.v_off;
    cd* RU = ws + ws_off[bi];
    cd* RV = RU + (int64_t)r * r;
    cd* M = RV + (int64_t)r * r;
    cd* X = M + (int64_t)r * r;
    int* srt_g = reinterpret_cast<int*>(X + (int64_t)r * r);
    auto qr = [&](cd* G, int len, cd* R) {
        if (len * r <= LDSC) {
            for (int e = tid; e < len * r; e += NTQ) lbuf[e] = G[e];
            __syncthreads();
            cgs2_qr<NTQ, QB>(lbuf, len, r, R, hbuf, red);
            for (int e = tid; e < len * r; e += NTQ) G[e] = lbuf[e];
            __syncthreads();
        } else {
            cgs2_qr<NTQ, QB>(G, len, r, R, hbuf, red);
        }
    };
    qr(U, t.m, RU);
    qr(V, t.n, RV);
    const bool core_lds = 2 * r * r <= LDSC;
    cd* Mw = core_lds ? lbuf : M;
    cd* Xw = core_lds ? lbuf + r * r : X;
    for (int e = tid; e < r * r; e += NTQ) {
        const int a = e % r, b = e / r;
        cd s = cmk(0.0, 0.0);
        // R_U upper triangular: l >= a; R_V: l >= b
        for (int l = max(a, b); l < r; ++l) s = cfma(RU[a + (int64_t)l * r], RV[b + (int64_t)l * r], s);
        Mw[e] = s;
        Xw[e] = cmk(a == b ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    jacobi_svd<NTQ>(Mw, Xw, r, &rot_flag);
    __syncthreads();
    if (core_lds)
        for (int e = tid; e < r * r; e += NTQ) {
            M[e] = Mw[e];
            X[e] = Xw[e];
        }
    for (int c = tid; c < r; c += NTQ) {
        double s = 0.0;
        for (int x = 0; x < r; ++x) s += cabs2(Mw[x + (int64_t)c * r]);
        sig[c] = sqrt(s);
    }
    __syncthreads();
    // rank sort: position of column c = #{d : sig[d] > sig[c] or (== and d < c)}
    for (int c = tid; c < r; c += NTQ) {
        int pos = 0;
        for (int d = 0; d < r; ++d) pos += (sig[d] > sig[c]) || (sig[d] == sig[c] && d < c);
        srt[pos] = c;
    }
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int c = 0; c < r; ++c) tot += sig[srt[c]] * sig[srt[c]];
        const double lim = eps * sqrt(tot);
        // smallest i with sqrt(sum_{l >= i} s_l^2) <= lim (the tail grows as i falls)
        double tail2 = 0.0;
        int keep = r;
        for (int i = r - 1; i >= 0; --i) {
            tail2 += sig[srt[i]] * sig[srt[i]];
            if (sqrt(tail2) <= lim) keep = i;
        }
        rank_out[bi] = keep;
    }
    for (int c = tid; c < r; c += NTQ) srt_g[c] = srt[c];
}

// Re-compression, phase B: write U' = Q_U M[:, srt[:r']] (m x r'
// column-major) and V' = X[:, srt[:r']]^H Q_V^T (r' x n row-major).
template <int NTQ>
__global__ void __launch_bounds__(NTQ)
k_recompress_b(const AcaTask* __restrict__ tasks, const int* __restrict__ order, const cd* __restrict__ scratch,
               const int* __restrict__ rank_in, const cd* __restrict__ ws, const int64_t* __restrict__ ws_off,
               const int* __restrict__ rank_new, cd* const* __restrict__ dst) {
    const int bi = order ? order[blockIdx.x] : (int)blockIdx.x;
    const AcaTask t = tasks[bi];
    const int r = rank_in[bi], rp = rank_new[bi];
    if (rp == 0) return;
    const int m = t.m, n = t.n;
    const cd* Q = scratch + t.u_off;
    const cd* Qv = scratch + t.v_off;
    const cd* M = ws + ws_off[bi] + 2 * (int64_t)r * r;
    const cd* X = M + (int64_t)r * r;
    const int* srt = reinterpret_cast<const int*>(X + (int64_t)r * r);
    cd* Uo = dst[bi];
    if (Uo == nullptr) return;   // block kept dense
    cd* Vo = Uo + (int64_t)m * rp;
    for (int e = threadIdx.x; e < m * rp; e += NTQ) {
        const int x = e % m, c = e / m;
        const cd* mc = M + (int64_t)srt[c] * r;
        cd s = cmk(0.0, 0.0);
        for (int l = 0; l < r; ++l) s = cfma(Q[(int64_t)l * m + x], mc[l], s);
        Uo[e] = s;
    }
    for (int e = threadIdx.x; e < rp * n; e += NTQ) {
        const int c = e / n, y = e % n;
        const cd* xc = X + (int64_t)srt[c] * r;
        cd s = cmk(0.0, 0.0);
        for (int l = 0; l < r; ++l) s = cfmac(xc[l], Qv[(int64_t)l * n + y], s);
        Vo[e] = s;
    }
}

// ---- launchers ----------------------------------------------------------------

void launch_near_assemble(const NearTask* tasks, int64_t ntasks, const double* pts, double k, double h,
                          cd* out, int* err, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_near_assemble, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, pts, k, h, out, err);
}

void launch_aca(bool dense, const AcaTask* tasks, const int* order, int64_t ntasks, const double* pts, double k,
                const cd* dense_src, cd* scratch, uint8_t* flags, double eps, int* rank_out, int* piv_log,
                int piv_stride, int* err, hipStream_t s) {
    if (ntasks == 0) return;
    if (dense)
        hipLaunchKernelGGL(k_aca<true>, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, order, pts, k, dense_src, scratch,
                           flags, eps, rank_out, piv_log, piv_stride, err);
    else
        hipLaunchKernelGGL(k_aca<false>, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, order, pts, k, dense_src, scratch,
                           flags, eps, rank_out, piv_log, piv_stride, err);
}

void launch_recompress_a(int kind, const AcaTask* tasks, const int* order, int64_t ntasks, cd* scratch,
                         const int* rank_in, cd* ws, const int64_t* ws_off, double eps, int* rank_out, hipStream_t s) {
    if (ntasks <= 0) return;
    if (kind == kRcWide)
        hipLaunchKernelGGL((k_recompress_a<NTW, kRcLdsWide, kQbWide>), dim3((unsigned)ntasks), dim3(NTW), 0, s, tasks, order,
                           scratch, rank_in, ws, ws_off, eps, rank_out);
    else if (kind == kRcSmall)
        hipLaunchKernelGGL((k_recompress_a<kWave, kRcLdsSmall, kQbSmall, kRcSmallLen>), dim3((unsigned)ntasks), dim3(kWave), 0, s, tasks,
                           order, scratch, rank_in, ws, ws_off, eps, rank_out);
    else
        hipLaunchKernelGGL((k_recompress_a<NTR, kRcLds, kQbRest>), dim3((unsigned)ntasks), dim3(NTR), 0, s, tasks, order, scratch,
                           rank_in, ws, ws_off, eps, rank_out);
}

void launch_recompress_b(int kind, const AcaTask* tasks, const int* order, int64_t ntasks, const cd* scratch,
                         const int* rank_in, const cd* ws, const int64_t* ws_off, const int* rank_new, cd* const* dst,
                         hipStream_t s) {
    if (ntasks <= 0) return;
    if (kind == kRcWide)
        hipLaunchKernelGGL(k_recompress_b<NTW>, dim3((unsigned)ntasks), dim3(NTW), 0, s, tasks, order, scratch, rank_in,
                           ws, ws_off, rank_new, dst);
    else if (kind == kRcSmall)
        hipLaunchKernelGGL(k_recompress_b<kWave>, dim3((unsigned)ntasks), dim3(kWave), 0, s, tasks, order, scratch,
                           rank_in, ws, ws_off, rank_new, dst);
    else
        hipLaunchKernelGGL(k_recompress_b<NTR>, dim3((unsigned)ntasks), dim3(NTR), 0, s, tasks, order, scratch, rank_in,
                           ws, ws_off, rank_new, dst);
}

}  // namespace hs
