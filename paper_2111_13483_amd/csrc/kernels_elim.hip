// The symmetric Schur elimination of the near field (Eq. 12-21, Sec. 3.2;
// the block inversion of Eq. 31-33, the coefficients of Eq. 34-37, the
// updates of Eq. 38-42), one step k after another. One kernel, k_elim_items,
// takes a list of work items, a workgroup each:
//
//   factor tile     W_kk^-1 by Gauss-Jordan (every tile of the step inverts
//                   the same block in its LDS, so the step needs no separate
//                   inversion launch), then its 64-column tile of
//                   alpha_kS = -W_kk^-1 W_kS over the panel of row k;
//   Schur tile      a 64 x 64 tile of the panel product W_kS^T alpha_kS,
//                   each element added to its target block W_ij (i <= j in S_k).
//
// With the look-ahead (kElimLook), step k's factor tiles first apply the
// previous step p's update of row k themselves (W_kj += W_pk^T alpha_pj), and
// p's Schur tiles skip that row, so one launch holds step k's factor tiles
// beside step p's Schur tiles: the inversion chain no longer waits for a
// Schur launch between two steps.
//
// Row k's pattern blocks W_kj (j in S_k ascending) lie back to back, each
// b_k x b_j row-major; read side by side they form a b_k x m panel whose
// column g is local column g - pcol[a] of the a-th block. alpha_kS has the
// same packing. The per-step pair table gives the offset of every target
// block; k_pair_table fills it from the filled pattern.
//
// The non-symmetric elimination that Sec. 3.2 compares against (Table 2)
// uses the same items on two entries per step (ElimStep flags): the left
// coefficients alpha'_ik = -W_ik W_kk^-1 are formed from the lower blocks,
// held transposed in a second copy of the upper layout, and both triangles
// receive their own Schur updates.
#include "devcommon.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int NTF = 512;            // the factor/alpha kernel: eight waves
constexpr int NWF = NTF / kWave;
constexpr int kLdc = kMaxLeaf + 1;   // column stride of the LDS inverse (odd: conflict-free column writes)
constexpr int kTile = 64;            // panel columns per factor tile; Schur tile width
constexpr int kTileR = kSchurRows;   // Schur tile height
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
// false if the block is singular (the error flag is raised). W_kk is read
// from LDS (row-major, stride b); it may share the result's storage, since
// every wave reads its columns before the first barrier.
template <int S, bool TWO>
__device__ __forceinline__ bool gj_invert(const cd* wkk, int b, int* err, cd* A, cd (*colbuf)[kMaxLeaf],
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
        a0[u] = wkk[(v0 ? r0 : 0) * b + jj];
        a1[u] = TWO ? wkk[(v1 ? r1 : 0) * b + jj] : cmk(0.0, 0.0);
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

// Register state of gj_invert_rot: slot u of lane (r, h) holds row r of a
// column of W_kk. The steps run as a loop over pairs whose pivot columns are
// always slot 0 (halves 0 and 1); after each pair the slots rotate down by
// one, so at pair t slot u holds column 2 ((u + t) mod U) + h, and every slot
// index is a constant without unrolling the steps.
template <int U>
struct GjRot {
    cd e[U];
    cd* rowx;
    cd* colx;
    int* err;
    int b, h, r, lane;
    int pos;     // position of this lane's row in the interchanged order
    int x0;      // source column tracker (column = lane)
    bool vr, used, ok;

    template <int HC>
    __device__ __forceinline__ void step(int C) {
        constexpr int un = HC == 0 ? 0 : (U > 1 ? 1 : 0);   // slot of column C + 1
        const cd ec = e[0];
        const double v = (h == HC && vr && !used) ? cabs2_exact(ec) : -1.0;
        const double vmax = wave_max_f64(v);
        if (!(vmax > 0.0)) {
            if (lane == 0) raise_err(err, vmax == 0.0 ? kErrSingular : kErrNumeric);
            ok = false;
            return;
        }
        unsigned long long m = __ballot(v == vmax);
        int q = __ffsll((long long)m) - 1;
        int qpos = __builtin_amdgcn_readlane(pos, q);
        m &= m - 1;
        while (m) {   // ties: lowest position
            const int l2 = __ffsll((long long)m) - 1;
            m &= m - 1;
            const int p2 = __builtin_amdgcn_readlane(pos, l2);
            if (p2 < qpos) { q = l2; qpos = p2; }
        }
        const bool isp = r == (q & 31);
        const cd inv = crecip(cmk(readlane_f64(ec.x, q), readlane_f64(ec.y, q)));
        // the pivot row (1 in column C) and column C, through LDS, by slot
        if (isp) {
#pragma unroll
            for (int u = 0; u < U; ++u) rowx[2 * u + h] = (u == 0 && h == HC) ? cmk(1.0, 0.0) : e[u];
        }
        if (h == HC) colx[r] = ec;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const cd f = colx[r];
        cd p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = rowx[2 * u + h];
        const cd gm = isp ? cmk(-inv.x, -inv.y) : cmul(f, inv);
        const double s = isp ? 0.0 : 1.0;
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int u = t == 0 ? un : (t <= un ? t - 1 : t);
            const double sv = (u == 0 && h == HC) ? 0.0 : s;
            const double ex = e[u].x * sv, ey = e[u].y * sv;
            e[u] = cmk(fma(-gm.x, p[u].x, fma(gm.y, p[u].y, ex)), fma(-gm.x, p[u].y, fma(-gm.y, p[u].x, ey)));
        }
        if (isp) used = true;
        pos = isp ? C : (pos == C ? qpos : pos);
        x0 = x0 == C ? qpos : (x0 == qpos ? C : x0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// Gauss-Jordan inversion of W_kk for b <= 2U <= 32 by wave 0 alone, with no
// barrier per pivot step: lane = row r (lane & 31) in half h (lane >> 5).
// W_kk is read from LDS (row-major, row stride ldi, possibly sharing A's
// storage: wave 0 holds it in registers before it writes A); the result goes
// to A column-major with column stride ldo. Pivot rule: the largest
// |a|^2 among the rows not yet eliminated, ties to the lowest position in the
// interchanged order; rows are not moved (each lane keeps its row's position
// and a used flag) and each column is stored by final position at the end,
// so the result and its layout match gj_invert. A pivot step is a wave max
// and ballot over column c, one exchange of the pivot row and of column c
// through LDS (in order within the wave), and the update e = s e - g p, where
// p is the pivot row (with 1 in column c), g the lane's multiplier over the
// pivot (the pivot row: -1/pivot) and s = 0 for the pivot row and for column
// c, else 1. One wave costs fewer cycles per pivot step than eight waves
// meeting at a barrier (measured: 35k against 41k cycles at b = 21). The
// other waves go straight to the closing barrier (or do other work first);
// *okf carries the outcome to them.
template <int U>
__device__ __forceinline__ bool gj_invert_rot(const cd* wkk, int b, int* err, cd* A, cd* rowx, cd* colx,
                                              int* srcmap, int* okf, int ldi, int ldo) {
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    if (wv == 0) {
        GjRot<U> g;
        g.rowx = rowx;
        g.colx = colx;
        g.err = err;
        g.b = b;
        g.lane = lane;
        g.h = lane >> 5;
        g.r = lane & 31;
        g.vr = g.r < b;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = 2 * u + g.h;
            g.e[u] = wkk[(g.vr ? g.r : 0) * ldi + (j < b ? j : 0)];
        }
        g.pos = g.r;
        g.x0 = lane;
        g.used = false;
        g.ok = true;
        for (int cp = 0; cp < b; cp += 2) {
            g.template step<0>(cp);
            if (!g.ok) break;
            if (cp + 1 < b) {
                g.template step<1>(cp + 1);
                if (!g.ok) break;
            }
            const cd t0 = g.e[0];
#pragma unroll
            for (int u = 0; u + 1 < U; ++u) g.e[u] = g.e[u + 1];
            g.e[U - 1] = t0;
        }
        if (g.ok) {
            const int T = (b + 1) / 2;   // rotations done
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = 2 * ((u + T) % U) + g.h;
                if (j < b && g.vr) A[j * ldo + g.pos] = g.e[u];
            }
            if (lane < b) srcmap[lane] = g.x0;
        }
        if (lane == 0) *okf = g.ok ? 1 : 0;
    }
    __syncthreads();
    return *okf != 0;
}


// gj_invert_rot with U chosen for b <= 32 (U = ceil(b / 2), rounded up to even)
__device__ __forceinline__ bool invert_small(const cd* src, int b, int* err, cd* out, cd* rowx, cd* colx, int* srcmap,
                                             int* okf, int ldi, int ldo) {
    const int need = (b + 1) / 2;
    if (need <= 2) return gj_invert_rot<2>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 4) return gj_invert_rot<4>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 6) return gj_invert_rot<6>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 8) return gj_invert_rot<8>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 10) return gj_invert_rot<10>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 12) return gj_invert_rot<12>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    if (need <= 14) return gj_invert_rot<14>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
    return gj_invert_rot<16>(src, b, err, out, rowx, colx, srcmap, okf, ldi, ldo);
}

namespace {

// Panels (W_kS, alpha_kS, W_kk and the look-ahead operands) are read and
// written through buffer resources on the step's own base pointer: 128-bit
// accesses, and an offset past the panel reads zero and writes nothing, so
// dead lanes need no branch. Every step's inputs come from earlier launches.
typedef int v4i __attribute__((ext_vector_type(4)));

// a wave-uniform value in a scalar register (the panels' bases and lengths
// are per step, the same in every lane)
__device__ __forceinline__ const cd* uniform_ptr(const cd* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const cd*>(((uint64_t)hi << 32) | lo);
}
struct Panel {
    __amdgpu_buffer_rsrc_t r;
    unsigned nbytes;   // n * 16 < 2^31 (the host bounds the panels)
    __device__ __forceinline__ Panel(const cd* p, int64_t n)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<cd*>(uniform_ptr(p)), (short)0,
                                              __builtin_amdgcn_readfirstlane((int)(n * 16)), 0x00020000)),
          nbytes((unsigned)__builtin_amdgcn_readfirstlane((int)(n * 16))) {}
    // byte offset of element i; outside [0, n) the panel's length, which the
    // range check rejects (loads read zero, stores are dropped)
    __device__ __forceinline__ unsigned off(int64_t i) const {
        return (i < 0 || i * 16 >= (int64_t)nbytes) ? nbytes : (unsigned)i * 16u;
    }
    __device__ __forceinline__ cd ld(int64_t i) const {
        const v4i v = __builtin_amdgcn_raw_buffer_load_b128(r, off(i), 0, 0);
        return cmk(__hiloint2double(v.y, v.x), __hiloint2double(v.w, v.z));
    }
    __device__ __forceinline__ void st(int64_t i, cd v) const {
        v4i w;
        w.x = __double2loint(v.x);
        w.y = __double2hiint(v.x);
        w.z = __double2loint(v.y);
        w.w = __double2hiint(v.y);
        __builtin_amdgcn_raw_buffer_store_b128(w, r, off(i), 0, 0);
    }
};

struct FactorSmem {
    cd A[kMaxLeaf * kLdc];      // W_kk (row-major, stride b), then its inverse (column-major, stride kLdc)
    cd colbuf[2][kMaxLeaf];
    cd pinv[2];
    int prow[4];
    int srcmap[kMaxLeaf];
    int pcol[kMaxPattern + 1];
    int cblk[kTile];
    int okf;
};
template <class A>
struct SchurSmem {
    A Xs[kKc][kTileR];
    A Ys[kKc][kTile];
    int rblk[kTileR], cblk[kTile];   // panel block of each tile row / column (-1 past the panel)
    int rst[kTileR], cst[kTile];     // its first panel column
    int rbj[kTileR], cbj[kTile];     // its width
};

// W_kk^-1 for 32 < b <= 64 by 2 x 2 blocks: with W_kk = [P Q; R T] (P of
// b1 = ceil(b / 2) rows), P^-1 and the inverse of the Schur complement
// T - R P^-1 Q each come from the single-wave Gauss-Jordan (partial pivoting
// within each half), joined by products in LDS:
//   E = P^-1 Q, F = R P^-1, H = (T - R E)^-1, G = E H,
//   W_kk^-1 = [P^-1 + G F, -G; -H F, H].
// Two inversions of b / 2 pivots cost less than one eight-wave inversion of
// b pivots (measured: 313k cycles at b = 64 for the latter). W_kk is in A
// (row-major, stride b); on return A holds W_kk^-1 column-major (stride
// kLdc) with srcmap the identity, the layout gj_invert leaves.
__device__ __forceinline__ bool invert_blocked(FactorSmem& sm, int b, int* err) {
    const int tid = threadIdx.x;
    const int b1 = (b + 1) / 2, b2 = b - b1;
    const int l1 = b1 + 1, l2 = b2 + 1;   // column strides of the half inverses
    cd* const M = sm.A;
    cd* const Po = sm.A + 4096;            // P^-1 by columns (b1 x l1)
    cd* const E = Po + 32 * 33;            // b1 x b2
    cd* const F = E + 32 * 32;             // b2 x b1
    cd* const Sc = F + 32 * 32;            // b2 x b2, then H by columns
    cd* const Ho = Sc + 32 * 32;           // b2 x l2
    int* const sp = sm.srcmap;
    int* const sh = sm.srcmap + 32;
    if (!invert_small(M, b1, err, Po, sm.colbuf[0], sm.colbuf[1], sp, &sm.okf, b, l1)) return false;
    // P^-1[i][j] = Po[sp[j] l1 + i]
    for (int e = tid; e < 2 * b1 * b2; e += NTF) {
        cd acc = cmk(0.0, 0.0);
        if (e < b1 * b2) {
            const int i = e / b2, j = e - (e / b2) * b2;
            for (int l = 0; l < b1; ++l) acc = cfma(Po[sp[l] * l1 + i], M[l * b + b1 + j], acc);
            E[e] = acc;
        } else {
            const int f = e - b1 * b2, i = f / b1, j = f - (f / b1) * b1;
            for (int l = 0; l < b1; ++l) acc = cfma(M[(b1 + i) * b + l], Po[sp[j] * l1 + l], acc);
            F[f] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < b2 * b2; e += NTF) {
        const int i = e / b2, j = e - (e / b2) * b2;
        cd acc = cmk(0.0, 0.0);
        for (int l = 0; l < b1; ++l) acc = cfma(M[(b1 + i) * b + l], E[l * b2 + j], acc);
        Sc[e] = csub(M[(b1 + i) * b + b1 + j], acc);
    }
    __syncthreads();
    if (!invert_small(Sc, b2, err, Ho, sm.colbuf[0], sm.colbuf[1], sh, &sm.okf, b2, l2)) return false;
    // H[i][j] = Ho[sh[j] l2 + i]; G = E H over M (no longer needed)
    cd* const G = M;
    for (int e = tid; e < b1 * b2; e += NTF) {
        const int i = e / b2, j = e - (e / b2) * b2;
        cd acc = cmk(0.0, 0.0);
        for (int k = 0; k < b2; ++k) acc = cfma(E[i * b2 + k], Ho[sh[j] * l2 + k], acc);
        G[e] = acc;
    }
    __syncthreads();
    constexpr int PT = 64 * 64 / NTF;
    cd v[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int e = tid + u * NTF;
        v[u] = cmk(0.0, 0.0);
        if (e < b * b) {
            const int i = e / b, j = e - (e / b) * b;
            if (i < b1 && j < b1) {
                cd acc = Po[sp[j] * l1 + i];
                for (int k = 0; k < b2; ++k) acc = cfma(G[i * b2 + k], F[k * b1 + j], acc);
                v[u] = acc;
            } else if (i < b1) {
                v[u] = cscale(G[i * b2 + (j - b1)], -1.0);
            } else if (j < b1) {
                cd acc = cmk(0.0, 0.0);
                for (int k = 0; k < b2; ++k) acc = cfma(Ho[sh[k] * l2 + (i - b1)], F[k * b1 + j], acc);
                v[u] = cscale(acc, -1.0);
            } else {
                v[u] = Ho[sh[j - b1] * l2 + (i - b1)];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int e = tid + u * NTF;
        if (e < b * b) {
            const int i = e / b, j = e - (e / b) * b;
            sm.A[j * kLdc + i] = v[u];
        }
    }
    if (tid < b) sm.srcmap[tid] = tid;
    __syncthreads();
    return true;
}

// The look-ahead update of one factor tile's columns (kElimLook):
// step k applies the previous step p's update of its own row, X_kg += W_pk^T
// alpha_pg (K = b_p) for every column g of the tile whose block is in S_p, in
// place in W; p's Schur tiles leave row k alone (kElimSkip0). Lane = column,
// waves w0, w0 + nw, ... take the rows; the product is accumulated from zero
// in ascending m and added once.
template <int QR>
__device__ __forceinline__ void lookahead_cols(const ElimStep& st, const ElimStep& ps, const FactorSmem& sm, int g0,
                                               int w0, int nw) {
    const int lane = threadIdx.x % kWave, g = g0 + lane;
    const int b = st.bk, bp = ps.bk;
    const Panel X(st.x, (int64_t)b * st.m), Wp(ps.x, (int64_t)bp * b), Ap(ps.y, (int64_t)bp * ps.m);
    const bool on = g < st.m;
    const int a = on ? sm.cblk[lane] : 0;
    const int pc = on ? gld(st.lamap + a) : -1;
    const bool up = pc >= 0;
    const int bj = sm.pcol[a + 1] - sm.pcol[a], lc = g - sm.pcol[a];
    const int64_t xg = (int64_t)b * sm.pcol[a] + lc;      // X[l][g] at xg + l bj
    const int64_t ag = up ? (int64_t)bp * pc + lc : -1;    // alpha_p[m][g'] at ag + m bj
    for (int l0 = w0; l0 < b; l0 += nw * QR) {
        cd acc[QR];
#pragma unroll
        for (int q = 0; q < QR; ++q) acc[q] = cmk(0.0, 0.0);
#pragma unroll 4
        for (int m = 0; m < bp; ++m) {
            const cd av = Ap.ld(up ? ag + (int64_t)m * bj : -1);
#pragma unroll
            for (int q = 0; q < QR; ++q) {
                const int l = l0 + nw * q;
                acc[q] = cfma(Wp.ld(l < b ? (int64_t)m * b + l : -1), av, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < QR; ++q) {
            const int l = l0 + nw * q;
            const int64_t i = (up && l < b) ? xg + (int64_t)l * bj : -1;
            const cd x = X.ld(i);
            X.st(i, cadd(x, acc[q]));
        }
    }
}

// 16 bytes per lane straight into LDS (lane l of the wave lands at
// dst_wave + 16 l); all such loads of a phase are in flight at once
__device__ __forceinline__ void load_lds16(const cd* src, cd* dst_wave) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                     (__attribute__((address_space(3))) void*)dst_wave, 16, 0, 0);
}
// n contiguous values from src into LDS dst (the whole workgroup)
__device__ __forceinline__ void stage_lds(const cd* src, int n, cd* dst) {
    const int tid = threadIdx.x, wb = tid - tid % kWave;
    for (int u = 0; u * NTF < n; ++u)
        if (u * NTF + tid < n) load_lds16(src + u * NTF + tid, dst + u * NTF + wb);
}

// LDS layout of the small factor tile (b <= 32) inside FactorSmem::A: W_kk
// and then its inverse at 0 (the inverse spans 32 kLdc values), the tile's X
// columns at kXo (row l at kXo + 64 l), the look-ahead operands W_pk and
// alpha_pk (b_p x b each, b_p <= 64) at kPo and kPo + 2048.
constexpr int kXo = 32 * kLdc;
constexpr int kPo = kXo + 32 * kTile;
static_assert(kPo + 2 * 64 * 32 <= kMaxLeaf * kLdc, "small factor tile layout");

// The factor tile for b <= 32 (and, with the look-ahead, b_p <= 64): every
// operand is staged into LDS by direct loads, so each phase waits for memory
// once. W_kk (and W_pk, alpha_pk) first; W_kk's look-ahead update is formed
// in LDS; wave 0 inverts while waves 1-7 bring the tile's X columns into LDS
// (with the look-ahead: X_kg + W_pk^T alpha_pg, also written back to W for
// the Schur tiles); then alpha = -W_kk^-1 X from LDS. Results as factor_tile.
__device__ __forceinline__ void factor_tile_small(const ElimStep& st, const ElimStep* ps, int ti, FactorSmem& sm) {
    const int b = st.bk, bp = ps ? ps->bk : 0;
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    cd* const A = sm.A;
    cd* const Xs = A + kXo;
    cd* const Wp = A + kPo;
    cd* const Ap = A + kPo + 2048;
    stage_lds(st.wkk, b * b, A);
    if (ps) {
        stage_lds(ps->x, bp * b, Wp);
        stage_lds(ps->y, bp * b, Ap);
    }
    for (int a = tid; a <= st.ne; a += NTF) sm.pcol[a] = gld(st.pcol + a);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int g0 = ti * kTile;
    for (int a = tid; a < st.ne; a += NTF) {
        const int lo = sm.pcol[a] > g0 ? sm.pcol[a] : g0;
        const int hi = sm.pcol[a + 1] < g0 + kTile ? sm.pcol[a + 1] : g0 + kTile;
        for (int g = lo; g < hi; ++g) sm.cblk[g - g0] = a;
    }
    // W_kk += W_pk^T alpha_pk (K = b_p), accumulated from zero in ascending m
    for (int e = tid; e < b * b; e += NTF) {
        const int i = e / b, j = e - (e / b) * b;
        cd v = A[e];
        if (ps) {
            cd acc = cmk(0.0, 0.0);
            for (int m = 0; m < bp; ++m) acc = cfma(Wp[m * b + i], Ap[m * b + j], acc);
            v = cadd(v, acc);
            A[e] = v;
        }
        if (ti == 0 && st.dfin) gst(st.dfin + e, v);
    }
    __syncthreads();
    // waves 1-7: the tile's X columns (rows l = w - 1 + 7 q) into LDS meanwhile
    const int g = g0 + lane;
    const bool on = g < st.m;
    const int a = on ? sm.cblk[lane] : 0;
    const int bj = sm.pcol[a + 1] - sm.pcol[a], lc = g - sm.pcol[a];
    const int64_t xg = (int64_t)b * sm.pcol[a] + lc;   // X[l][g] at xg + l bj
    if (wv > 0) {
        const Panel X(st.x, (int64_t)b * st.m);
        const int pc = (ps && on) ? gld(st.lamap + a) : -1;
        if (ps) {
            const Panel Apn(ps->y, (int64_t)bp * ps->m);
            const int64_t ag = pc >= 0 ? (int64_t)bp * pc + lc : -1;   // alpha_p[m][g'] at ag + m bj
            constexpr int QR = 5;   // rows per wave: 7 waves x 5 >= 32
            cd acc[QR];
#pragma unroll
            for (int q = 0; q < QR; ++q) acc[q] = cmk(0.0, 0.0);
#pragma unroll 8
            for (int m = 0; m < bp; ++m) {
                const cd av = Apn.ld(ag >= 0 ? ag + (int64_t)m * bj : -1);
#pragma unroll
                for (int q = 0; q < QR; ++q) {
                    const int l = wv - 1 + 7 * q;
                    if (l < b) acc[q] = cfma(Wp[m * b + l], av, acc[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < QR; ++q) {
                const int l = wv - 1 + 7 * q;
                if (l < b) {
                    const int64_t i = on ? xg + (int64_t)l * bj : -1;
                    cd x = X.ld(i);
                    if (pc >= 0) {
                        x = cadd(x, acc[q]);
                        X.st(i, x);
                    }
                    Xs[l * kTile + lane] = x;
                }
            }
        } else {
            for (int l = wv - 1; l < b; l += NWF - 1) Xs[l * kTile + lane] = X.ld(on ? xg + (int64_t)l * bj : -1);
        }
    }
    const bool ok = invert_small(A, b, st.err, A, sm.colbuf[0], sm.colbuf[1], sm.srcmap, &sm.okf, b, kLdc);
    if (!ok) return;
    const bool tr = (st.flags & kElimTrans) != 0;
    if (ti == 0 && !tr)
        for (int e = tid; e < b * b; e += NTF) {
            const int i = e / b, j = e - (e / b) * b;
            gst(st.dinv + e, A[sm.srcmap[j] * kLdc + i]);
        }
    if (!on) return;
    // alpha tile from LDS: Y[r][g] = -sum_l W_kk^-1[r][l] X[l][g] (kElimTrans:
    // W_kk^-1[l][r]); lane = column, wave = rows wv, wv + 8, ...
    constexpr int RW = 4;   // 8 waves x 4 >= 32
    cd acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) acc[q] = cmk(0.0, 0.0);
    int srow[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + NWF * q;
        srow[q] = r < b ? sm.srcmap[r] * kLdc : 0;
    }
    for (int l = 0; l < b; ++l) {
        const cd xv = Xs[l * kTile + lane];
        if (!tr) {
            const cd* dcol = A + sm.srcmap[l] * kLdc;
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int r = wv + NWF * q;
                if (r < b) acc[q] = cfma(dcol[r], xv, acc[q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int r = wv + NWF * q;
                if (r < b) acc[q] = cfma(A[srow[q] + l], xv, acc[q]);
            }
        }
    }
    const Panel Y(st.y, (int64_t)b * st.m);
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + NWF * q;
        if (r < b) Y.st(xg + (int64_t)r * bj, cscale(acc[q], -1.0));
    }
}

// One factor tile: W_kk^-1 by Gauss-Jordan (every tile of the step inverts
// the same block), tile 0 writes D_k^-1, then the tile's 64 columns of
// alpha_kS = -W_kk^-1 W_kS. ps (kElimLook) is the previous step of the
// component, whose update of row k this tile applies first: to W_kk in LDS
// and to its own panel columns in W (waves 1-7 while wave 0 inverts, for b <=
// 32); the final W_kk then exists only in LDS, and tile 0 keeps it at
// st.dfin when that is set.
__device__ __forceinline__ void factor_tile(const ElimStep& st, const ElimStep* ps, int ti, FactorSmem& sm) {
    const int b = st.bk;
    const int tid = threadIdx.x, lane = tid % kWave;
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    for (int a = tid; a <= st.ne; a += NTF) sm.pcol[a] = gld(st.pcol + a);
    __syncthreads();
    // panel block of each column of this tile: every block marks its span
    const int g0 = ti * kTile;
    for (int a = tid; a < st.ne; a += NTF) {
        const int lo = sm.pcol[a] > g0 ? sm.pcol[a] : g0;
        const int hi = sm.pcol[a + 1] < g0 + kTile ? sm.pcol[a + 1] : g0 + kTile;
        for (int g = lo; g < hi; ++g) sm.cblk[g - g0] = a;
    }
    // W_kk (with the look-ahead: plus W_pk^T alpha_pk, K = b_p) into LDS
    const Panel Wkk(st.wkk, (int64_t)b * b);
    for (int e = tid; e < b * b; e += NTF) {
        const int i = e / b, j = e - (e / b) * b;
        cd v = Wkk.ld(e);
        if (ps) {
            const Panel Wp(ps->x, (int64_t)ps->bk * b), Ap(ps->y, (int64_t)ps->bk * ps->m);
            cd acc = cmk(0.0, 0.0);
#pragma unroll 4
            for (int m = 0; m < ps->bk; ++m) acc = cfma(Wp.ld((int64_t)m * b + i), Ap.ld((int64_t)m * b + j), acc);
            v = cadd(v, acc);
        }
        sm.A[e] = v;
        if (ti == 0 && st.dfin) gst(st.dfin + e, v);
    }
    __syncthreads();
    bool ok;
    if (b <= 32) {
        if (ps && wv > 0) lookahead_cols<(32 + NWF - 2) / (NWF - 1)>(st, *ps, sm, g0, wv - 1, NWF - 1);
        ok = invert_small(sm.A, b, st.err, sm.A, sm.colbuf[0], sm.colbuf[1], sm.srcmap, &sm.okf, b, kLdc);
    } else if (b <= 64) {
        ok = invert_blocked(sm, b, st.err);
        if (ps) {
            lookahead_cols<4>(st, *ps, sm, g0, wv, NWF);
            __syncthreads();
        }
    } else {
        ok = gj_invert<(kMaxLeaf + NWF - 1) / NWF, true>(sm.A, b, st.err, sm.A, sm.colbuf, sm.pinv, sm.prow,
                                                         sm.srcmap);
        if (ps) {
            lookahead_cols<4>(st, *ps, sm, g0, wv, NWF);
            __syncthreads();
        }
    }
    if (!ok) return;
    const bool tr = (st.flags & kElimTrans) != 0;
    // W_kk^-1[i][j] = A[srcmap[j]][i] (column srcmap[j] of the LDS result)
    if (ti == 0 && !tr)
        for (int e = tid; e < b * b; e += NTF) {
            const int i = e / b, j = e - (e / b) * b;
            gst(st.dinv + e, sm.A[sm.srcmap[j] * kLdc + i]);
        }
    // alpha tile: Y[r][g] = -sum_l W_kk^-1[r][l] X[l][g] (kElimTrans: W_kk^-1[l][r]),
    // lane = column, wave = rows wv, wv + 8, ...
    const Panel X(st.x, (int64_t)b * st.m), Y(st.y, (int64_t)b * st.m);
    const int g = g0 + lane;
    const bool on = g < st.m;
    const int a = on ? sm.cblk[lane] : 0;
    const int bj = sm.pcol[a + 1] - sm.pcol[a];
    const int64_t off = on ? (int64_t)b * sm.pcol[a] + (g - sm.pcol[a]) : -1;
    constexpr int RW = (kMaxLeaf + NWF - 1) / NWF;
    cd acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) acc[q] = cmk(0.0, 0.0);
    constexpr int LB = 16;
    // this wave's rows r read column srcmap[r] (kElimTrans) or the columns srcmap[l] of A
    int srow[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + NWF * q;
        srow[q] = r < b ? sm.srcmap[r] * kLdc : 0;
    }
    for (int l0 = 0; l0 < b; l0 += LB) {
        cd xv[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) xv[u] = X.ld(on && l0 + u < b ? off + (int64_t)(l0 + u) * bj : -1);
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int l = l0 + u;
            if (l >= b) break;
            if (!tr) {
                const cd* dcol = sm.A + sm.srcmap[l] * kLdc;
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = wv + NWF * q;
                    if (r < b) acc[q] = cfma(dcol[r], xv[u], acc[q]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const int r = wv + NWF * q;
                    if (r < b) acc[q] = cfma(sm.A[srow[q] + l], xv[u], acc[q]);
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + NWF * q;
        if (r < b) Y.st(on ? off + (int64_t)r * bj : -1, cscale(acc[q], -1.0));
    }
}

// One kTileR x 64 tile (ti, tj) of C = Xs_kS^T alpha_kS (K = b_k; Xs = W for the
// symmetric elimination) by NTS threads, each element (p, q) with block(p) <=
// block(q) (kElimStrict: <) added to its target block; kElimSkip0 leaves the
// rows of block 0 to the next step's look-ahead. A = cd: FP64 products; A =
// cf (mixed-precision setups): the panel tiles are rounded to complex64 and
// the product is formed and accumulated in FP32, then added to the FP64
// target once.
template <class A, int NTS>
__device__ __forceinline__ void schur_tile(const ElimStep& st, int ti, int tj, SchurSmem<A>& sm) {
    constexpr int RPT = kTileR * 16 / NTS;   // rows per thread (columns: 4)
    const int kk = st.bk, m = st.m, ne = st.ne;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int gr = ti * kTileR, gc = tj * kTile;
    const bool strict = (st.flags & kElimStrict) != 0;
    const bool skip0 = (st.flags & kElimSkip0) != 0;
    if (tid < kTileR) sm.rblk[tid] = -1;
    if (tid < kTile) sm.cblk[tid] = -1;
    __syncthreads();
    // every block marks its span in the row tile and in the column tile
    for (int a = tid; a < ne; a += NTS) {
        const int p0 = gld(st.pcol + a), p1 = gld(st.pcol + a + 1);
        for (int g = (p0 > gr ? p0 : gr); g < (p1 < gr + kTileR ? p1 : gr + kTileR); ++g) {
            sm.rblk[g - gr] = a; sm.rst[g - gr] = p0; sm.rbj[g - gr] = p1 - p0;
        }
        for (int g = (p0 > gc ? p0 : gc); g < (p1 < gc + kTile ? p1 : gc + kTile); ++g) {
            sm.cblk[g - gc] = a; sm.cst[g - gc] = p0; sm.cbj[g - gc] = p1 - p0;
        }
    }
    __syncthreads();
    // target of (p, q): W + pair[tri(a_p, a_q)] + (local row) * b_q + (local
    // column). Targets lie in later block rows than the panels and belong to
    // this tile alone, so they are read before the product is formed.
    int64_t dst[RPT][4];
    bool live[RPT][4];
    {
        int ap[RPT], lr[RPT], aq[4], lc[4], bq[4];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int pr = ty * RPT + i;
            ap[i] = sm.rblk[pr];
            lr[i] = gr + pr - sm.rst[pr];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int qc = tx * 4 + j;
            aq[j] = sm.cblk[qc];
            lc[j] = gc + qc - sm.cst[qc];
            bq[j] = sm.cbj[qc];
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int64_t tbase = (int64_t)ap[i] * ne - (int64_t)ap[i] * (ap[i] - 1) / 2 - ap[i];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // aq = -1 past the panel
                live[i][j] = ap[i] >= 0 && (strict ? aq[j] > ap[i] : aq[j] >= ap[i]) && !(skip0 && ap[i] == 0);
                dst[i][j] = gld(st.pair + (live[i][j] ? tbase + aq[j] : 0));
            }
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[i][j] = live[i][j] ? dst[i][j] + (int64_t)lr[i] * bq[j] + lc[j] : 0;
    }
    // staging: thread tid always serves row-tile column tid % kTileR (K rows
    // tid / kTileR + (NTS / kTileR) u) and column-tile column tid % 64 (K rows
    // tid / 64 + (NTS / 64) u)
    constexpr int SUX = kKc * kTileR / NTS, SRX = NTS / kTileR;
    constexpr int SU = kKc * kTile / NTS, SR = NTS / kTile;
    const int cx = tid % kTileR, lx = tid / kTileR;
    const int c = tid % kTile, l0 = tid / kTile;
    const int ra = sm.rblk[cx], ca = sm.cblk[c];
    const int64_t ro = ra >= 0 ? (int64_t)kk * sm.rst[cx] + (gr + cx - sm.rst[cx]) : 0;
    const int64_t co = ca >= 0 ? (int64_t)kk * sm.cst[c] + (gc + c - sm.cst[c]) : 0;
    const int rb = sm.rbj[cx], cbw = sm.cbj[c];
    const Panel Xp(st.xs, (int64_t)kk * m), Yp(st.y, (int64_t)kk * m);
    cd acc[RPT][4];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = gld(st.w + dst[i][j]);
    // the product is accumulated from zero in ascending l and added once
    A prod[RPT][4];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) prod[i][j] = czero<A>();
    for (int k0 = 0; k0 < kk; k0 += kKc) {
        cd xv[SUX], yv[SU];
#pragma unroll
        for (int u = 0; u < SUX; ++u) {
            const int gl = k0 + lx + SRX * u;
            xv[u] = Xp.ld((gl < kk && ra >= 0) ? ro + (int64_t)gl * rb : -1);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int gl = k0 + l0 + SR * u;
            yv[u] = Yp.ld((gl < kk && ca >= 0) ? co + (int64_t)gl * cbw : -1);
        }
        if (k0 > 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < SUX; ++u) sm.Xs[lx + SRX * u][cx] = to_arith<A>(xv[u]);
#pragma unroll
        for (int u = 0; u < SU; ++u) sm.Ys[l0 + SR * u][c] = to_arith<A>(yv[u]);
        __syncthreads();
        const int lend = kk - k0 < kKc ? kk - k0 : kKc;
        for (int l = 0; l < lend; ++l) {
            A av[RPT], bv[4];
#pragma unroll
            for (int i = 0; i < RPT; ++i) av[i] = sm.Xs[l][ty * RPT + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sm.Ys[l][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) prod[i][j] = cfma(av[i], bv[j], prod[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (live[i][j]) gst(st.w + dst[i][j], cadd(acc[i][j], to_cd(prod[i][j])));
}

}  // namespace

// One elimination launch: a workgroup per item, a factor tile (tj < 0: ti is
// its panel tile) or a Schur tile. A launch holds the factor tiles of some
// steps and the Schur tiles of others; every item's inputs were written by
// earlier launches (the host's grouping).
template <class A>
__global__ void __launch_bounds__(NTF) k_elim_items(const ElimStep* __restrict__ steps,
                                                    const ElimTile* __restrict__ items) {
    constexpr size_t kBytes = sizeof(FactorSmem) > sizeof(SchurSmem<A>) ? sizeof(FactorSmem) : sizeof(SchurSmem<A>);
    __shared__ __attribute__((aligned(16))) unsigned char raw[kBytes];
    const ElimTile it = items[blockIdx.x];
    const ElimStep& st = steps[it.step];
    if (it.tj < 0) {
        const ElimStep* ps = (st.flags & kElimLook) ? &steps[st.prev] : nullptr;
        if (st.bk <= 32 && (!ps || ps->bk <= 64))
            factor_tile_small(st, ps, it.ti, *reinterpret_cast<FactorSmem*>(raw));
        else factor_tile(st, ps, it.ti, *reinterpret_cast<FactorSmem*>(raw));
    } else {
        schur_tile<A, NTF>(st, it.ti, it.tj, *reinterpret_cast<SchurSmem<A>*>(raw));
    }
}

void launch_pair_table(const PairStep* steps, int64_t nsteps, int* err, hipStream_t s) {
    if (nsteps > 0) hipLaunchKernelGGL(k_pair_table, dim3((unsigned)nsteps), dim3(NT), 0, s, steps, err);
}

void launch_elim_items(const ElimStep* steps, const ElimTile* items, int64_t nitems, bool fp32, hipStream_t s) {
    if (nitems <= 0) return;
    if (fp32) hipLaunchKernelGGL(k_elim_items<cf>, dim3((unsigned)nitems), dim3(NTF), 0, s, steps, items);
    else hipLaunchKernelGGL(k_elim_items<cd>, dim3((unsigned)nitems), dim3(NTF), 0, s, steps, items);
}

}  // namespace hs
