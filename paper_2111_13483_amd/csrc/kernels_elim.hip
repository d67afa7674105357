// The symmetric Schur elimination of the near field (Eq. 12-21, Sec. 3.2;
// the block inversion of Eq. 31-33, the coefficients of Eq. 34-37, the
// updates of Eq. 38-42), one step k after another, two launches per step:
//
//   k_factor_alpha  W_kk^-1 by Gauss-Jordan (every workgroup of the step
//                   inverts the same block in its LDS, so the step needs no
//                   separate inversion launch), then its 64-column tile of
//                   alpha_kS = -W_kk^-1 W_kS over the panel of row k;
//   k_schur_tiles   64 x 64 tiles of the panel product W_kS^T alpha_kS,
//                   each element added to its target block W_ij (i <= j in S_k).
//
// Row k's pattern blocks W_kj (j in S_k ascending) lie back to back, each
// b_k x b_j row-major; read side by side they form a b_k x m panel whose
// column g is local column g - pcol[a] of the a-th block. alpha_kS has the
// same packing. The per-step pair table gives the offset of every target
// block; k_pair_table fills it from the filled pattern.
//
// The non-symmetric elimination that Sec. 3.2 compares against (Table 2)
// uses the same two kernels on two entries per step (ElimStep flags): the
// left coefficients alpha'_ik = -W_ik W_kk^-1 are formed from the lower
// blocks, held transposed in a second copy of the upper layout, and both
// triangles receive their own Schur updates.
#include "devcommon.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int NTF = 512;            // the factor/alpha kernel: eight waves
constexpr int NWF = NTF / kWave;
constexpr int kLdc = kMaxLeaf + 1;   // column stride of the LDS inverse (odd: conflict-free column writes)
constexpr int kTile = 64;            // panel tile edge
constexpr int kKc = 32;              // K chunk of the Schur tiles

// loads and stores through global-address-space pointers (global_* rather
// than flat_* instructions, so waits count only memory operations)
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
typedef double v2d __attribute__((ext_vector_type(2)));
template <>
__device__ __forceinline__ cd gld<cd>(const cd* p) {
    const v2d v = *(const __attribute__((address_space(1))) v2d*)p;
    return cmk(v.x, v.y);
}
__device__ __forceinline__ void gst(cd* p, cd v) {
    v2d t;
    t.x = v.x;
    t.y = v.y;
    *(__attribute__((address_space(1))) v2d*)p = t;
}

}  // namespace

// Offsets of the Schur targets of every step: pair[tri(a, b)] for a <= b < ne
// is the W offset of block (S_k[a], S_k[b]): the diagonal block when a == b,
// else the entry of S_k[b] in row S_k[a] of the filled pattern (present
// because the pattern is closed under elimination, Sec. 3.3).
__global__ void __launch_bounds__(NT) k_pair_table(const PairStep* __restrict__ steps, int* err) {
    const PairStep ps = steps[blockIdx.x];
    const int ne = ps.ne;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int a = wv; a < ne; a += NT / kWave) {
        const int i = ps.sk[a];
        const int64_t base = (int64_t)a * ne - (int64_t)a * (a - 1) / 2 - a;
        const int r0 = ps.rowptr[i], r1 = ps.rowptr[i + 1];
        for (int b = a + lane; b < ne; b += kWave) {
            int64_t off;
            if (b == a) {
                off = ps.wd_off[i];
            } else {
                const int j = ps.sk[b];
                int lo = r0, hi = r1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (ps.cols[mid] < j) lo = mid + 1;
                    else hi = mid;
                }
                if (lo == r1 || ps.cols[lo] != j) {
                    raise_err(err, kErrNumeric);
                    off = 0;
                } else {
                    off = ps.w_off[lo];
                }
            }
            ps.pair[base + b] = off;
        }
    }
}

// 1 / a as conj(a) / |a|^2: one division (pivots are far from the
// overflow and underflow ranges)
__device__ __forceinline__ cd crecip(cd a) {
    const double r = 1.0 / cabs2_exact(a);
    return cmk(a.x * r, -a.y * r);
}

// maximum over the wave (NaN ignored unless every lane holds one)
__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fmax(v, dpp_f64<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fmax(v, dpp_f64<0x124>(v));   // row_ror:4
    v = fmax(v, dpp_f64<0x128>(v));   // row_ror:8
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Pivot row of a column held as (row lane, value n0) and (row lane + 64, n1):
// largest |a|^2 among rows lo..b-1, ties to the lowest row. Returns the row,
// or -1 (all zero: singular) / -2 (no finite candidate).
__device__ __forceinline__ int pivot_row(cd n0, cd n1, int lo, int b, bool two) {
    const int lane = threadIdx.x % kWave;
    const int r0 = lane, r1 = lane + kWave;
    double v0 = (r0 >= lo && r0 < b) ? cabs2_exact(n0) : -1.0;
    const double v1 = (two && r1 >= lo && r1 < b) ? cabs2_exact(n1) : -1.0;
    const bool pick1 = v1 > v0;
    const double v = pick1 ? v1 : v0;
    const double vmax = wave_max_f64(v);
    if (!(vmax > 0.0)) return vmax == 0.0 ? -1 : -2;
    const unsigned long long m0 = __ballot(v == vmax && !pick1);
    if (m0) return __ffsll((long long)m0) - 1;
    return __ffsll((long long)__ballot(v == vmax)) - 1 + kWave;
}

// Gauss-Jordan inversion of W_kk with partial pivoting (row pivot: largest
// |a|^2 among the rows not yet eliminated, ties to the lowest row; rows
// interchanged as they are chosen, columns interchanged back at the end).
// The block lives in registers: wave w holds columns w, w + 8, ... (S slots),
// lane r rows r and r + 64 (TWO), so row interchanges and the pivot row are
// read across lanes. In step c the wave holding column c + 1 publishes it
// (the multipliers of the next step), finds the next pivot in it and
// publishes the pivot row and its reciprocal: a step costs one exchange
// through LDS and one barrier. On return the eliminated block is in LDS
// (column-major, stride kLdc) and srcmap holds the column interchanges;
// false if the block is singular (the error flag is raised).
template <int S, bool TWO>
__device__ __forceinline__ bool gj_invert(const cd* __restrict__ wkk, int b, int* err, cd* A, cd (*colbuf)[kMaxLeaf],
                                          cd* pinv, int* prow, int* srcmap) {
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int r0 = lane, r1 = lane + kWave;
    const bool v0 = r0 < b, v1 = TWO && r1 < b;
    cd a0[S], a1[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const int j = wv + NWF * u;
        const int jj = j < b ? j : 0;
        a0[u] = gld(wkk + (v0 ? r0 : 0) * b + jj);
        a1[u] = TWO ? gld(wkk + (v1 ? r1 : 0) * b + jj) : cmk(0.0, 0.0);
    }
    int x0 = lane, x1 = lane + kWave;   // source column trackers of the final column interchanges
    auto publish = [&](int jn, cd e0, cd e1) {
        cd* nb = colbuf[jn & 1];
        if (v0) nb[r0] = e0;
        if (v1) nb[r1] = e1;
        const int q = pivot_row(e0, e1, jn, b, TWO);
        cd qinv = cmk(0.0, 0.0);
        if (q >= 0)
            qinv = crecip(q < kWave ? cmk(readlane_f64(e0.x, q), readlane_f64(e0.y, q))
                                    : cmk(readlane_f64(e1.x, q - kWave), readlane_f64(e1.y, q - kWave)));
        if (lane == 0) {
            prow[jn & 1] = q;
            pinv[jn & 1] = qinv;
        }
    };
    if (wv == 0) publish(0, a0[0], a1[0]);
    __syncthreads();
    for (int c = 0; c < b; ++c) {
        const int p = __builtin_amdgcn_readfirstlane(prow[c & 1]);
        const cd inv = pinv[c & 1];
        if (p < 0) {
            if (tid == 0) raise_err(err, p == -1 ? kErrSingular : kErrNumeric);
            return false;   // every wave reads the same pivot
        }
        const cd* cb = colbuf[c & 1];
        // after interchanging rows c and p, row r holds what row srow(r) held
        const int s0 = r0 == c ? p : (r0 == p ? c : r0);
        const int s1 = r1 == c ? p : (r1 == p ? c : r1);
        const cd f0 = v0 ? cb[s0] : cmk(0.0, 0.0);
        const cd f1 = v1 ? cb[s1] : cmk(0.0, 0.0);
        x0 = x0 == c ? p : (x0 == p ? c : x0);
        x1 = x1 == c ? p : (x1 == p ? c : x1);
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int j = wv + NWF * u;
            cd& e0 = a0[u];
            cd& e1 = a1[u];
            const cd pv = (!TWO || p < kWave) ? cmk(readlane_f64(e0.x, p), readlane_f64(e0.y, p))
                                              : cmk(readlane_f64(e1.x, p - kWave), readlane_f64(e1.y, p - kWave));
            const cd cv = (!TWO || c < kWave) ? cmk(readlane_f64(e0.x, c), readlane_f64(e0.y, c))
                                              : cmk(readlane_f64(e1.x, c - kWave), readlane_f64(e1.y, c - kWave));
            const cd o0 = r0 == c ? pv : (r0 == p ? cv : e0);
            const cd o1 = r1 == c ? pv : (r1 == p ? cv : e1);
            const cd pjs = (j == c) ? inv : cmul(pv, inv);
            cd n0, n1;
            if (r0 == c) n0 = pjs;
            else if (j == c) n0 = cmk(-(f0.x * inv.x - f0.y * inv.y), -(f0.x * inv.y + f0.y * inv.x));
            else n0 = csub(o0, cmul(f0, pjs));
            if (r1 == c) n1 = pjs;
            else if (j == c) n1 = cmk(-(f1.x * inv.x - f1.y * inv.y), -(f1.x * inv.y + f1.y * inv.x));
            else n1 = csub(o1, cmul(f1, pjs));
            e0 = n0;
            if (TWO) e1 = n1;
        }
        const int jn = c + 1;
        if (jn < b && jn % NWF == wv) {
            // the next pivot column, picked out of the slots
            const int un = jn / NWF;
            cd e0 = a0[0], e1 = a1[0];
#pragma unroll
            for (int u = 1; u < S; ++u)
                if (u == un) {
                    e0 = a0[u];
                    e1 = a1[u];
                }
            publish(jn, e0, e1);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const int j = wv + NWF * u;
        if (j < b) {
            if (v0) A[j * kLdc + r0] = a0[u];
            if (v1) A[j * kLdc + r1] = a1[u];
        }
    }
    if (wv == 0) {
        if (lane < b) srcmap[lane] = x0;
        if (lane + kWave < b) srcmap[lane + kWave] = x1;
    }
    __syncthreads();
    return true;
}

// The same inversion for b <= 32, two columns per register: half h of a wave
// (32 lanes, lane = row) holds one column, wave w columns 16u + 2w + h. Rows
// are not moved: each lane keeps its row's position in the interchanged
// order and a used flag, the pivot is the largest |a|^2 among unused rows
// with ties to the lowest position (the row the interchanging algorithm
// picks), and each column is stored by final position at the end, so the
// result and its layout match gj_invert.
template <int S>
__device__ __forceinline__ bool gj_invert_half(const cd* __restrict__ wkk, int b, int* err, cd* A,
                                               cd (*colbuf)[kMaxLeaf], cd* pinv, int* prow, int* srcmap) {
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int h = lane >> 5, r = lane & 31;
    const bool vr = r < b;
    cd e[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const int j = 16 * u + 2 * wv + h;
        e[u] = gld(wkk + (vr ? r : 0) * b + (j < b ? j : 0));
    }
    int pos = r;           // position of this lane's row in the interchanged order
    bool used = false;
    int x0 = lane;         // source column tracker of the final column interchanges (column = lane)
    // the wave holding column jn publishes it, picks the next pivot and its
    // reciprocal; slot layout: prow[2 * (jn & 1)] = row, [+1] = its position
    auto publish = [&](int jn, cd ev) {
        const int hn = jn & 1;
        cd* nb = colbuf[jn & 1];
        if (h == hn && vr) nb[r] = ev;
        const double v = (h == hn && vr && !used) ? cabs2_exact(ev) : -1.0;
        const double vmax = wave_max_f64(v);
        int q = -2;
        if (vmax > 0.0) {
            unsigned long long m = __ballot(v == vmax);
            q = __ffsll((long long)m) - 1;
            m &= m - 1;
            if (m) {   // ties: lowest position
                int qpos = __builtin_amdgcn_readlane(pos, q);
                while (m) {
                    const int l2 = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int p2 = __builtin_amdgcn_readlane(pos, l2);
                    if (p2 < qpos) { q = l2; qpos = p2; }
                }
            }
        } else if (vmax == 0.0) {
            q = -1;
        }
        cd qinv = cmk(0.0, 0.0);
        int qpos = 0;
        if (q >= 0) {
            qinv = crecip(cmk(readlane_f64(ev.x, q), readlane_f64(ev.y, q)));
            qpos = __builtin_amdgcn_readlane(pos, q);
        }
        if (lane == 0) {
            prow[2 * (jn & 1)] = q < 0 ? q : q - 32 * hn;
            prow[2 * (jn & 1) + 1] = qpos;
            pinv[jn & 1] = qinv;
        }
    };
    if (wv == 0) publish(0, e[0]);
    __syncthreads();
    for (int c = 0; c < b; ++c) {
        const int p = __builtin_amdgcn_readfirstlane(prow[2 * (c & 1)]);
        const int pp = __builtin_amdgcn_readfirstlane(prow[2 * (c & 1) + 1]);
        const cd inv = pinv[c & 1];
        if (p < 0) {
            if (tid == 0) raise_err(err, p == -1 ? kErrSingular : kErrNumeric);
            return false;
        }
        const cd f = vr ? colbuf[c & 1][r] : cmk(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const int j = 16 * u + 2 * wv + h;
            // the pivot row's entry of this lane's column
            const double p0x = readlane_f64(e[u].x, p), p0y = readlane_f64(e[u].y, p);
            const double p1x = readlane_f64(e[u].x, p + 32), p1y = readlane_f64(e[u].y, p + 32);
            const cd pv = h ? cmk(p1x, p1y) : cmk(p0x, p0y);
            const cd pjs = (j == c) ? inv : cmul(pv, inv);
            if (r == p) e[u] = pjs;
            else if (j == c) e[u] = cmk(-(f.x * inv.x - f.y * inv.y), -(f.x * inv.y + f.y * inv.x));
            else e[u] = csub(e[u], cmul(f, pjs));
        }
        // row p becomes position c; the row at position c takes p's position
        if (r == p) used = true;
        pos = (r == p) ? c : (pos == c ? pp : pos);
        x0 = x0 == c ? pp : (x0 == pp ? c : x0);
        const int jn = c + 1;
        if (jn < b && (jn % 16) / 2 == wv) {
            const int un = jn / 16;
            cd ev = e[0];
#pragma unroll
            for (int u = 1; u < S; ++u)
                if (u == un) ev = e[u];
            publish(jn, ev);
        }
        __syncthreads();
    }
    // columns stored by final position
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const int j = 16 * u + 2 * wv + h;
        if (j < b && vr) A[j * kLdc + pos] = e[u];
    }
    if (wv == 0 && lane < b) srcmap[lane] = x0;
    __syncthreads();
    return true;
}

// W_kk^-1 (Gauss-Jordan above), then one 64-column tile of alpha.
__global__ void __launch_bounds__(NTF) k_factor_alpha(const ElimStep* __restrict__ steps,
                                                      const ElimTile* __restrict__ tiles) {
    const ElimTile tl = tiles[blockIdx.x];
    const ElimStep st = steps[tl.step];
    const int b = st.bk;
    __shared__ cd A[kMaxLeaf * kLdc];
    __shared__ cd colbuf[2][kMaxLeaf];
    __shared__ cd pinv[2];
    __shared__ int prow[4];
    __shared__ int srcmap[kMaxLeaf];
    __shared__ int pcol[kMaxPattern + 1];
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    for (int a = tid; a <= st.ne; a += NTF) pcol[a] = gld(st.pcol + a);
    bool ok;
    if (b <= 16) ok = gj_invert_half<1>(st.wkk, b, st.err, A, colbuf, pinv, prow, srcmap);
    else if (b <= 32) ok = gj_invert_half<2>(st.wkk, b, st.err, A, colbuf, pinv, prow, srcmap);
    else if (b <= kWave) ok = gj_invert<8, false>(st.wkk, b, st.err, A, colbuf, pinv, prow, srcmap);
    else ok = gj_invert<(kMaxLeaf + NWF - 1) / NWF, true>(st.wkk, b, st.err, A, colbuf, pinv, prow, srcmap);
    if (!ok) return;
    const bool tr = (st.flags & kElimTrans) != 0;
    // W_kk^-1[i][j] = A[i][srcmap[j]]
    if (tl.ti == 0 && !tr)
        for (int e = tid; e < b * b; e += NTF) {
            const int i = e / b, j = e - (e / b) * b;
            gst(st.dinv + e, A[srcmap[j] * kLdc + i]);
        }
    // panel block of each column of this tile: every block marks its span
    __shared__ int cblk[kTile];
    const int g0 = tl.ti * kTile;
    for (int a = tid; a < st.ne; a += NTF) {
        const int lo = pcol[a] > g0 ? pcol[a] : g0, hi = pcol[a + 1] < g0 + kTile ? pcol[a + 1] : g0 + kTile;
        for (int g = lo; g < hi; ++g) cblk[g - g0] = a;
    }
    __syncthreads();
    // alpha tile: Y[r][g] = -sum_l W_kk^-1[r][l] X[l][g] (kElimTrans: W_kk^-1[l][r]),
    // lane = column, wave = rows wv, wv + 8, ...
    const int g = g0 + lane;
    if (g >= st.m) return;
    const int a = cblk[lane];
    const int bj = pcol[a + 1] - pcol[a];
    const int64_t off = (int64_t)b * pcol[a] + (g - pcol[a]);
    const cd* xg = st.x + off;
    cd* yg = st.y + off;
    constexpr int RW = (kMaxLeaf + NWF - 1) / NWF;
    cd acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) acc[q] = cmk(0.0, 0.0);
    constexpr int LB = 16;
    if (!tr) {
        for (int l0 = 0; l0 < b; l0 += LB) {
            cd xv[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) xv[u] = gld(xg + (int64_t)(l0 + u < b ? l0 + u : b - 1) * bj);
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int l = l0 + u;
                if (l >= b) break;
                const cd* dcol = A + srcmap[l] * kLdc;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = wv + NWF * q;
                    if (r < b) acc[q] = cfma(dcol[r], xv[u], acc[q]);
                }
            }
        }
    } else {
        // W_kk^-1[l][r] = A[srcmap[r] * kLdc + l]: this wave's rows r fix the columns of A it reads
        int srow[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int r = wv + NWF * q;
            srow[q] = r < b ? srcmap[r] * kLdc : 0;
        }
        for (int l0 = 0; l0 < b; l0 += LB) {
            cd xv[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) xv[u] = gld(xg + (int64_t)(l0 + u < b ? l0 + u : b - 1) * bj);
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int l = l0 + u;
                if (l >= b) break;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = wv + NWF * q;
                    if (r < b) acc[q] = cfma(A[srow[q] + l], xv[u], acc[q]);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + NWF * q;
        if (r < b) gst(yg + (int64_t)r * bj, cscale(acc[q], -1.0));
    }
}

// One 64 x 64 tile (ti, tj) of C = Xs_kS^T alpha_kS (K = b_k; Xs = W for the
// symmetric elimination), each element (p, q) with block(p) <= block(q)
// (kElimStrict: <) added to its target block.
// A = cd: FP64 products; A = cf (mixed-precision setups): the panel tiles
// are rounded to complex64 and the product is formed and accumulated in
// FP32, then added to the FP64 target once.
template <class A>
__global__ void __launch_bounds__(NT) k_schur_tiles(const ElimStep* __restrict__ steps,
                                                    const ElimTile* __restrict__ tiles) {
    const ElimTile tl = tiles[blockIdx.x];
    const ElimStep st = steps[tl.step];
    const int kk = st.bk, m = st.m, ne = st.ne;
    __shared__ A Xs[kKc][kTile];
    __shared__ A Ys[kKc][kTile];
    __shared__ int rblk[kTile], cblk[kTile];   // panel block of each tile row / column (-1 past the panel)
    __shared__ int rst[kTile], cst[kTile];     // its first panel column
    __shared__ int rbj[kTile], cbj[kTile];     // its width
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int gr = tl.ti * kTile, gc = tl.tj * kTile;
    const bool strict = (st.flags & kElimStrict) != 0;
    if (tid < kTile) { rblk[tid] = -1; cblk[tid] = -1; }
    __syncthreads();
    // every block marks its span in the row tile and in the column tile
    for (int a = tid; a < ne; a += NT) {
        const int p0 = gld(st.pcol + a), p1 = gld(st.pcol + a + 1);
        for (int g = (p0 > gr ? p0 : gr); g < (p1 < gr + kTile ? p1 : gr + kTile); ++g) {
            rblk[g - gr] = a; rst[g - gr] = p0; rbj[g - gr] = p1 - p0;
        }
        for (int g = (p0 > gc ? p0 : gc); g < (p1 < gc + kTile ? p1 : gc + kTile); ++g) {
            cblk[g - gc] = a; cst[g - gc] = p0; cbj[g - gc] = p1 - p0;
        }
    }
    __syncthreads();
    // target of (p, q): W + pair[tri(a_p, a_q)] + (local row) * b_q + (local
    // column). Targets lie in later block rows than the panels and belong to
    // this tile alone, so they are read before the product is formed.
    int64_t dst[4][4];
    bool live[4][4];
    {
        int ap[4], lr[4], aq[4], lc[4], bq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pr = ty * 4 + i, qc = tx * 4 + i;
            ap[i] = rblk[pr];
            lr[i] = gr + pr - rst[pr];
            aq[i] = cblk[qc];
            lc[i] = gc + qc - cst[qc];
            bq[i] = cbj[qc];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t tbase = (int64_t)ap[i] * ne - (int64_t)ap[i] * (ap[i] - 1) / 2 - ap[i];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                live[i][j] = ap[i] >= 0 && (strict ? aq[j] > ap[i] : aq[j] >= ap[i]);   // aq = -1 past the panel
                dst[i][j] = gld(st.pair + (live[i][j] ? tbase + aq[j] : 0));
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[i][j] = live[i][j] ? dst[i][j] + (int64_t)lr[i] * bq[j] + lc[j] : 0;
    }
    cd acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = gld(st.w + dst[i][j]);
    // staging: thread tid always serves panel column tid % 64 of both tiles,
    // rows tid / 64 + 4 u of the K chunk
    constexpr int SU = kKc * kTile / NT;
    const int c = tid % kTile, l0 = tid / kTile;
    const int ra = rblk[c], ca = cblk[c];
    const int64_t ro = ra >= 0 ? (int64_t)kk * rst[c] + (gr + c - rst[c]) : 0;
    const int64_t co = ca >= 0 ? (int64_t)kk * cst[c] + (gc + c - cst[c]) : 0;
    const int rb = rbj[c], cbw = cbj[c];
    // the product is accumulated from zero in ascending l and added once
    A prod[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) prod[i][j] = czero<A>();
    for (int k0 = 0; k0 < kk; k0 += kKc) {
        cd xv[SU], yv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int gl = k0 + l0 + 4 * u;
            const bool ok = gl < kk;
            xv[u] = gld(st.xs + ((ok && ra >= 0) ? ro + (int64_t)gl * rb : 0));
            yv[u] = gld(st.y + ((ok && ca >= 0) ? co + (int64_t)gl * cbw : 0));
        }
        if (k0 > 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int gl = k0 + l0 + 4 * u;
            const bool ok = gl < kk;
            Xs[l0 + 4 * u][c] = (ok && ra >= 0) ? to_arith<A>(xv[u]) : czero<A>();
            Ys[l0 + 4 * u][c] = (ok && ca >= 0) ? to_arith<A>(yv[u]) : czero<A>();
        }
        __syncthreads();
        const int lend = kk - k0 < kKc ? kk - k0 : kKc;
        for (int l = 0; l < lend; ++l) {
            A av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = Xs[l][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Ys[l][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) prod[i][j] = cfma(av[i], bv[j], prod[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (live[i][j]) gst(st.w + dst[i][j], cadd(acc[i][j], to_cd(prod[i][j])));
}

void launch_pair_table(const PairStep* steps, int64_t nsteps, int* err, hipStream_t s) {
    if (nsteps > 0) hipLaunchKernelGGL(k_pair_table, dim3((unsigned)nsteps), dim3(NT), 0, s, steps, err);
}

void launch_factor_alpha(const ElimStep* steps, const ElimTile* tiles, int64_t ntiles, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_factor_alpha, dim3((unsigned)ntiles), dim3(NTF), 0, s, steps, tiles);
}

void launch_schur_tiles(const ElimStep* steps, const ElimTile* tiles, int64_t ntiles, bool fp32, hipStream_t s) {
    if (ntiles <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_schur_tiles<cf>, dim3((unsigned)ntiles), dim3(NT), 0, s, steps, tiles);
    else hipLaunchKernelGGL(k_schur_tiles<cd>, dim3((unsigned)ntiles), dim3(NT), 0, s, steps, tiles);
}

}  // namespace hs
