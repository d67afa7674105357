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
#include "devcommon.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int kLdc = kMaxLeaf + 1;   // column stride of the LDS inverse (odd: conflict-free column writes)
constexpr int kTile = 64;            // panel tile edge
constexpr int kKc = 32;              // K chunk of the Schur tiles

// panel column g -> (block a, local column) by binary search over pcol[0..ne]
__device__ __forceinline__ int panel_block(const int* pcol, int ne, int g) {
    int lo = 0, hi = ne - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pcol[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
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

// Gauss-Jordan inversion of W_kk with partial pivoting (row pivot: largest
// |a|^2 among the rows not yet eliminated, ties to the lowest row; rows
// interchanged as they are chosen, columns interchanged back at the end),
// then one tile of alpha. The block sits column-major in LDS; lane r of every
// wave owns rows r and r + 64, the four waves take the columns in turn. The
// pivot column of the next step is copied aside as it is produced, so a step
// needs one barrier: every wave finds the pivot itself from that copy.
__global__ void __launch_bounds__(NT) k_factor_alpha(const ElimStep* __restrict__ steps,
                                                     const ElimTile* __restrict__ tiles) {
    const ElimTile tl = tiles[blockIdx.x];
    const ElimStep st = steps[tl.step];
    const int b = st.bk;
    __shared__ cd A[kMaxLeaf * kLdc];
    __shared__ cd colbuf[2][kMaxLeaf];
    __shared__ int srcmap[kMaxLeaf];
    __shared__ int pcol[kMaxPattern + 1];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    for (int e = tid; e < b * b; e += NT) {
        const int i = e / b, j = e - (e / b) * b;
        const cd v = st.wkk[e];
        A[j * kLdc + i] = v;
        if (j == 0) colbuf[0][i] = v;
    }
    for (int a = tid; a <= st.ne; a += NT) pcol[a] = st.pcol[a];
    const int r0 = lane, r1 = lane + kWave;
    const bool two = b > kWave;
    int x0 = lane, x1 = lane + kWave;   // source column trackers of the final column interchanges
    __syncthreads();
    for (int c = 0; c < b; ++c) {
        const cd* cb = colbuf[c & 1];
        ArgMax am{-1.0, 0x7fffffff};
        if (r0 >= c && r0 < b) am = ArgMax{cabs2_exact(cb[r0]), r0};
        if (two && r1 >= c && r1 < b) am = amax_pick(am, ArgMax{cabs2_exact(cb[r1]), r1});
        am = wave_argmax(am);
        const int p = am.i;
        if (!(am.v > 0.0)) {
            if (tid == 0) raise_err(st.err, am.v == 0.0 ? kErrSingular : kErrNumeric);
            return;   // every wave takes the same decision
        }
        const cd inv = cdiv(cmk(1.0, 0.0), cb[p]);
        // after interchanging rows c and p, row r holds what row srow(r) held
        const int s0 = r0 == c ? p : (r0 == p ? c : r0);
        const int s1 = r1 == c ? p : (r1 == p ? c : r1);
        const cd f0 = cb[s0 < b ? s0 : 0];
        const cd f1 = two ? cb[s1 < b ? s1 : 0] : cmk(0.0, 0.0);
        x0 = x0 == c ? p : (x0 == p ? c : x0);
        x1 = x1 == c ? p : (x1 == p ? c : x1);
        cd* nb = colbuf[(c + 1) & 1];
        for (int j = wv; j < b; j += NT / kWave) {
            cd* col = A + j * kLdc;
            // every read of this column before any write to it
            const cd pj = col[p];
            const cd o0 = col[s0 < b ? s0 : 0];
            const cd o1 = two ? col[s1 < b ? s1 : 0] : cmk(0.0, 0.0);
            const cd pjs = (j == c) ? inv : cmul(pj, inv);
            cd n0, n1;
            if (r0 == c) n0 = pjs;
            else if (j == c) n0 = cmk(-(f0.x * inv.x - f0.y * inv.y), -(f0.x * inv.y + f0.y * inv.x));
            else n0 = csub(o0, cmul(f0, pjs));
            if (r1 == c) n1 = pjs;
            else if (j == c) n1 = cmk(-(f1.x * inv.x - f1.y * inv.y), -(f1.x * inv.y + f1.y * inv.x));
            else n1 = csub(o1, cmul(f1, pjs));
            if (r0 < b) {
                col[r0] = n0;
                if (j == c + 1) nb[r0] = n0;
            }
            if (two && r1 < b) {
                col[r1] = n1;
                if (j == c + 1) nb[r1] = n1;
            }
        }
        __syncthreads();
    }
    if (wv == 0) {
        if (r0 < b) srcmap[r0] = x0;
        if (two && r1 < b) srcmap[r1] = x1;
    }
    __syncthreads();
    // W_kk^-1[i][j] = A[i][srcmap[j]]
    if (tl.ti == 0)
        for (int e = tid; e < b * b; e += NT) {
            const int i = e / b, j = e - (e / b) * b;
            st.dinv[e] = A[srcmap[j] * kLdc + i];
        }
    // alpha tile: Y[r][g] = -sum_l W_kk^-1[r][l] X[l][g], lane = column, wave = rows wv, wv + 4, ...
    const int g = tl.ti * kTile + lane;
    if (g >= st.m) return;
    const int a = panel_block(pcol, st.ne, g);
    const int bj = pcol[a + 1] - pcol[a];
    const int64_t off = (int64_t)b * pcol[a] + (g - pcol[a]);
    const cd* xg = st.x + off;
    cd* yg = st.y + off;
    constexpr int RW = (kMaxLeaf + 3) / 4;
    cd acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) acc[q] = cmk(0.0, 0.0);
    constexpr int LB = 16;
    for (int l0 = 0; l0 < b; l0 += LB) {
        cd xv[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) xv[u] = (l0 + u < b) ? xg[(int64_t)(l0 + u) * bj] : cmk(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int l = l0 + u;
            if (l >= b) break;
            const cd* dcol = A + srcmap[l] * kLdc;
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int r = wv + 4 * q;
                if (r < b) acc[q] = cfma(dcol[r], xv[u], acc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int r = wv + 4 * q;
        if (r < b) yg[(int64_t)r * bj] = cscale(acc[q], -1.0);
    }
}

// One 64 x 64 tile (ti, tj) of C = W_kS^T alpha_kS (K = b_k), each element
// (p, q) with block(p) <= block(q) added to its target block.
__global__ void __launch_bounds__(NT) k_schur_tiles(const ElimStep* __restrict__ steps,
                                                    const ElimTile* __restrict__ tiles) {
    const ElimTile tl = tiles[blockIdx.x];
    const ElimStep st = steps[tl.step];
    const int kk = st.bk, m = st.m, ne = st.ne;
    __shared__ cd Xs[kKc][kTile];
    __shared__ cd Ys[kKc][kTile];
    __shared__ int pcol[kMaxPattern + 1];
    __shared__ int rblk[kTile], cblk[kTile];
    __shared__ int64_t roff[kTile], coff[kTile];
    __shared__ int rbj[kTile], cbj[kTile];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    for (int a = tid; a <= ne; a += NT) pcol[a] = st.pcol[a];
    __syncthreads();
    if (tid < 2 * kTile) {
        const int c = tid % kTile;
        const int g = (tid < kTile ? tl.ti : tl.tj) * kTile + c;
        int a = -1, bj = 0;
        int64_t off = 0;
        if (g < m) {
            a = panel_block(pcol, ne, g);
            bj = pcol[a + 1] - pcol[a];
            off = (int64_t)kk * pcol[a] + (g - pcol[a]);
        }
        if (tid < kTile) { rblk[c] = a; rbj[c] = bj; roff[c] = off; }
        else { cblk[c] = a; cbj[c] = bj; coff[c] = off; }
    }
    cd acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cmk(0.0, 0.0);
    for (int k0 = 0; k0 < kk; k0 += kKc) {
        __syncthreads();
        for (int e = tid; e < kKc * kTile; e += NT) {
            const int l = e / kTile, c = e % kTile, gl = k0 + l;
            cd xv = cmk(0.0, 0.0), yv = cmk(0.0, 0.0);
            if (gl < kk) {
                if (rblk[c] >= 0) xv = st.x[roff[c] + (int64_t)gl * rbj[c]];
                if (cblk[c] >= 0) yv = st.y[coff[c] + (int64_t)gl * cbj[c]];
            }
            Xs[l][c] = xv;
            Ys[l][c] = yv;
        }
        __syncthreads();
        const int lend = kk - k0 < kKc ? kk - k0 : kKc;
        for (int l = 0; l < lend; ++l) {
            cd av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = Xs[l][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Ys[l][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = cfma(av[i], bv[j], acc[i][j]);
        }
    }
    // target of (p, q): W + pair[tri(a_p, a_q)] + (local row) * b_q + (local column)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int pr = ty * 4 + i;
        const int ap = rblk[pr];
        if (ap < 0) continue;
        const int lr = tl.ti * kTile + pr - pcol[ap];
        const int64_t tbase = (int64_t)ap * ne - (int64_t)ap * (ap - 1) / 2 - ap;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int qc = tx * 4 + j;
            const int aq = cblk[qc];
            if (aq < ap) continue;   // also skips columns past the panel (aq = -1)
            const int lc = tl.tj * kTile + qc - pcol[aq];
            cd* dst = st.w + st.pair[tbase + aq] + (int64_t)lr * cbj[qc] + lc;
            *dst = cadd(*dst, acc[i][j]);
        }
    }
}

void launch_pair_table(const PairStep* steps, int64_t nsteps, int* err, hipStream_t s) {
    if (nsteps > 0) hipLaunchKernelGGL(k_pair_table, dim3((unsigned)nsteps), dim3(NT), 0, s, steps, err);
}

void launch_factor_alpha(const ElimStep* steps, const ElimTile* tiles, int64_t ntiles, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_factor_alpha, dim3((unsigned)ntiles), dim3(NT), 0, s, steps, tiles);
}

void launch_schur_tiles(const ElimStep* steps, const ElimTile* tiles, int64_t ntiles, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_schur_tiles, dim3((unsigned)ntiles), dim3(NT), 0, s, steps, tiles);
}

}  // namespace hs
