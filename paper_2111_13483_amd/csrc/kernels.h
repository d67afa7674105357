// Task descriptors and launchers of the gfx950 kernels (host-visible).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hs {

typedef double2 cd;
typedef float2 cf;

constexpr int kMaxRankCap = 256;   // largest ACA rank a block may reach
// device error flag bits
enum : int { kErrSingular = 1, kErrNumeric = 2, kErrRankCap = 4, kErrCoincident = 8 };

constexpr int kMaxLeaf = 96;       // largest leaf block the dense kernels take (LDS bound)
constexpr int kMaxPattern = 1024;  // longest row of the filled pattern the elimination takes
constexpr int kSchurRows = 128;    // Schur tiles of the elimination: kSchurRows x 64 panel columns

// Per-column GMRES state on the device.
struct ColState {
    double bnorm;         // ||b||
    double beta;          // norm of the cycle's starting residual
    double relres;        // true relative residual at the last cycle end
    double tol;
    int32_t active;       // 1 while the column takes inner steps in this cycle
    int32_t steps;        // inner steps in the current cycle
    int32_t total;        // inner steps overall
    int32_t done;         // 1 once the column has stopped for good
    int32_t budget;       // max inner steps overall
    int32_t fixed;        // 1: ignore the inner tolerance test
    int32_t pad0, pad1;
};
// Which right-hand-side columns a matvec or sweep launch computes: all
// (mode 0), those still taking steps in the cycle (1: active), or those that
// took steps in it (2: steps > 0). Skipped columns' outputs are left as they
// were; every counter of a sweep advances as usual.
struct ColMask {
    const ColState* st;
    int32_t mode;
    int32_t pad;
};
__device__ __forceinline__ bool col_live(const ColMask& m, int c) {
    if (m.mode == 0) return true;
    return m.mode == 1 ? m.st[c].active != 0 : m.st[c].steps > 0;
}
__device__ __forceinline__ bool cols_live(const ColMask& m, int c0, int cs) {
    bool any = false;
    for (int c = 0; c < cs; ++c) any |= col_live(m, c0 + c);
    return any;
}

// One stored near block Z_ij (i <= j): b_i x b_j row-major at `off`.
struct NearTask {
    int64_t off;
    int32_t i0, m;        // tree-order start and size of leaf i (rows)
    int32_t j0, n;        // tree-order start and size of leaf j (columns)
};

// One block to compress with ACA: rows t0..t0+m, columns s0..s0+n (points),
// or a dense m x n row-major source at src_off.
struct AcaTask {
    int64_t src_off;
    int32_t t0, m, s0, n;
    int32_t cap;          // rank cap of this block
    int32_t pad;
    int64_t u_off, v_off; // scratch element offsets of U (m x cap) and V (cap x n)
    int64_t flag_off;     // byte offset of m + n "used" flags
};

// Copy a (possibly transposed) block or zero it: dst (rows x cols row-major).
struct CopyTask {
    int64_t dst_off, src_off;   // src_off < 0: zero fill
    int32_t rows, cols;
    int32_t transpose;          // 1: dst[a][b] = src[b][a] (src is cols x rows)
    int32_t dst_ld;             // row stride of dst (0: cols)
};

// C (m x n) = beta_acc ? C + sign * op(A) B : sign * op(A) B, all row-major;
// op(A)[a][l] = transA ? A[l][a] (A stored kk x m) : A[a][l] (A stored m x kk).
struct GemmTask {
    int64_t c_off, a_off, b_off;
    int32_t m, n, kk;
    int32_t pad;
};

// One far entry of a sweep: alpha block at aoff (dense if rank < 0, else
// U V), source and target blocks, slot base (times nrhs) of its result.
struct PushEnt {
    int64_t aoff, slot;
    int32_t src, dst, rank, pad;
};

// Low-rank or dense operator block of the sweeps / matvec.
struct SweepEnt {
    int64_t off;          // element offset into the alpha store
    int32_t k;            // the other block index
    int32_t rank;         // -1: dense
};

// Gather contribution: y[seg + a, c] += slot[s * base + off + a + c * len]
struct GatherEnt {
    int64_t base;         // slot start for one right-hand side (scaled by s)
    int32_t len;          // slot length (column stride within the slot)
    int32_t off;          // offset of this leaf inside the slot
};

// ---- build ----
void launch_near_assemble(const NearTask* tasks, int64_t ntasks, const double* pts, double k, double h, cd* out,
                          int* err, hipStream_t s);
// ACA of every block, one workgroup each; workgroup w takes block order[w]
// (null: w).
void launch_aca(bool dense, const AcaTask* tasks, const int* order, int64_t ntasks, const double* pts, double k,
                const cd* dense_src, cd* scratch, uint8_t* flags, double eps, int* rank_out, int* piv_log,
                int piv_stride, int* err, hipStream_t s);
// Re-compression of the listed blocks, one workgroup each; workgroup w takes
// block order[w] (null: w). kind kRcWide: 1024-thread workgroups with a
// 64 KB LDS buffer, for the blocks of rank above kRcWideRank (their QR dot
// products and Jacobi pairs spread over 16 waves); kRcRest: 256 threads and
// 8 KB; kRcSmall: one wave and 16 KB, for lists of blocks of at most
// kRcSmallLen points a side (the fill-in blocks of leaves up to 64 points).
constexpr int kRcWideRank = 32;
constexpr int kRcSmallLen = 64;
enum { kRcRest = 0, kRcWide = 1, kRcSmall = 2 };
void launch_recompress_a(int kind, const AcaTask* tasks, const int* order, int64_t ntasks, cd* scratch,
                         const int* rank_in, cd* ws, const int64_t* ws_off, double eps, int* rank_out, hipStream_t s);
void launch_recompress_b(int kind, const AcaTask* tasks, const int* order, int64_t ntasks, const cd* scratch,
                         const int* rank_in, const cd* ws, const int64_t* ws_off, const int* rank_new, cd* const* dst,
                         hipStream_t s);

// ---- setup ----
// Contiguous copies from scattered device sources: dst[dst_off + e] = src[e], e < count.
struct PtrCopy {
    const cd* src;
    int64_t dst_off;
    int64_t count;
};
void launch_copy_ptrs(const PtrCopy* tasks, int64_t ntasks, cd* dst, hipStream_t s);
// dst (rows x cols row-major, at dst_off) = the rows x cols column-major
// matrix at src (a low-rank factor U laid into a row-major panel)
struct ColMajorCopy {
    const cd* src;
    int64_t dst_off;
    int32_t rows, cols;
};
void launch_copy_colmajor(const ColMajorCopy* tasks, int64_t ntasks, cd* dst, hipStream_t s);
// Setup-side low-rank arithmetic: base[dst_off] (ba x bb row-major) +=
// L^T T R with T = base[t_off] (ta x tb row-major), L = va (ra x ba
// row-major, ta = ra) or the identity (va null, ta = ba), and R = vb (rb x
// bb row-major, tb = rb) or the identity (vb null, tb = bb).
struct CoreExpandTask {
    const cd* va;
    const cd* vb;
    int64_t dst_off, t_off;
    int32_t ba, bb, ra, rb;
};
void launch_core_expand(const CoreExpandTask* tasks, int64_t ntasks, cd* base, hipStream_t s);
void launch_copy_blocks(const CopyTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s);
// One elimination step k of one geometry (Eq. 14, 19). The pattern blocks
// W_kj of row k (j in S_k ascending) lie back to back at x, b_k x b_j each,
// row-major; alpha_kj gets the same packing at y. Panel column g (< m) of the
// step is local column g - pcol[a] of block a, pcol[a] <= g < pcol[a + 1].
// pair[tri(a, b)], a <= b < ne, row-major over the upper triangle, is the
// offset from w of target block (S_k[a], S_k[b]).
struct ElimStep {
    const cd* wkk;         // W_kk, b_k x b_k row-major
    cd* dinv;              // W_kk^-1 (out)
    const cd* x;           // W_kS panel: the factor kernel's right-hand side
    const cd* xs;          // the panel whose transpose is the Schur product's left operand
    cd* y;                 // alpha_kS panel (out)
    cd* w;                 // base of the Schur targets
    const int64_t* pair;   // ne (ne + 1) / 2 target offsets
    const int32_t* pcol;   // ne + 1 panel column starts
    int* err;              // device error flag of the geometry
    int32_t bk, ne, m, flags;
    // look-ahead (kElimLook):
    cd* dfin;              // the final W_kk, written by factor tile 0 (null: left in W)
    const int32_t* lamap;  // per block a of S_k, its first column in the previous step's panel (-1: absent)
    int32_t prev;          // entry of the previous step of the same component (-1: none)
    int32_t pad;
};
// ElimStep flags. Symmetric elimination: none (xs = x). The non-symmetric
// elimination (Sec. 3.2's comparator) runs two entries per step:
//   upper: x = W_kS, xs = Wt_kS (the lower blocks W_ik stored transposed in
//          the upper layout), y = alpha_kS; targets W_ab += W_ak alpha_kb, a <= b;
//   lower: x = Wt_kS with kElimTrans (y = -W_kk^-T Wt_kS = alpha'_Sk^T), xs =
//          W_kS; targets Wt_ab += W_ka^T y_kb (kElimStrict: a < b only).
constexpr int32_t kElimTrans = 1;    // factor: y = -W_kk^-T x, and D^-1 is not written
constexpr int32_t kElimStrict = 2;   // Schur: only targets with block(row) < block(column)
// Look-ahead (symmetric elimination): when S_p of the previous step p of the
// component starts with k, step k's factor tiles apply p's update of row k
// themselves (kElimLook on k) and p's Schur tiles skip the rows of their
// block 0 (kElimSkip0 on p), so step k's factor tiles and p's Schur tiles can
// share a launch.
constexpr int32_t kElimLook = 4;
constexpr int32_t kElimSkip0 = 8;
// One workgroup's share of a step: panel column tile ti (factor/alpha, 64
// columns) or output tile (ti, tj) (Schur update: panel rows kSchurRows ti ..,
// columns 64 tj ..).
struct ElimTile {
    int32_t step;
    int16_t ti, tj;
};
// Input of the pair tables: S_k (ne entries) and the filled pattern in CSR
// with the W offsets of its blocks.
struct PairStep {
    const int32_t* sk;
    const int32_t* rowptr;
    const int32_t* cols;
    const int64_t* w_off;
    const int64_t* wd_off;
    int64_t* pair;
    int32_t ne, pad;
};
void launch_pair_table(const PairStep* steps, int64_t nsteps, int* err, hipStream_t s);
// One elimination launch over items (tj < 0: a factor tile, ti its panel
// tile; else Schur tile (ti, tj)) whose inputs earlier launches wrote. fp32:
// the Schur products in complex64 with FP32 accumulation (mixed-precision
// setups).
void launch_elim_items(const ElimStep* steps, const ElimTile* items, int64_t nitems, bool fp32, hipStream_t s);
// Chunk products M = L C of the sweep plan, by 64 x 64 output tiles: one
// entry per row of a chunk (A row at a_off, nonzero over chunk columns
// [k0, k0 + kw), output row at c_off) and one per tile (chunk, first row,
// rows, first column).
struct ChunkRow {
    int64_t a_off, c_off;
    int32_t k0, kw;
};
struct ChunkTile {
    int64_t b_off;        // the chunk's C (csize x width, row-major)
    int32_t row0, nrow;   // chunk rows [row0, row0 + nrow) as ChunkRow indices
    int32_t col0, width;  // output columns [col0, col0 + 64) of width
    int32_t kmin, kmax;   // union of the rows' column ranges
};
void launch_chunk_gemm(const ChunkTile* tiles, int64_t ntiles, const ChunkRow* rows, const cd* A, const cd* B, cd* C,
                       hipStream_t s);
void launch_gemm(const GemmTask* tasks, int64_t ntasks, const cd* A, const cd* B, cd* C, bool transA, bool accumulate,
                 double sign, hipStream_t s);

// ---- solve ----
void launch_permute(const cd* src, cd* dst, const int64_t* perm, int64_t n, int64_t nrhs, bool to_tree,
                    hipStream_t s);
// Near and far parts of the matvec from complex128 or complex64 matrix
// copies (vectors and accumulation in complex128 either way).
void launch_near_mv(const ColMask& mk, const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const cd* Z,
                    const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s);
void launch_near_mv(const ColMask& mk, const NearTask* tasks, const int64_t* slot_base, int64_t ntasks, const cf* Z,
                    const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s);
// Far tasks [0, nwg) take one workgroup each; tasks [nwg, ntasks) have at
// most 64 x 64 points and rank <= kFarWaveRank and take one wave each.
constexpr int kFarWaveRank = 16;
void launch_far_mv(const ColMask& mk, const AcaTask* geom, const int* rank, cd* const* uv, const int64_t* slot_base,
                   int64_t nwg, int64_t ntasks, const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s);
void launch_far_mv(const ColMask& mk, const AcaTask* geom, const int* rank, cf* const* uv, const int64_t* slot_base,
                   int64_t nwg, int64_t ntasks, const cd* x, int64_t n, int nrhs, cd* slots, hipStream_t s);
// complex128 -> complex64 copies: dst[dst_off + e] = src[e], e < count
void launch_to_c64(const PtrCopy* tasks, int64_t ntasks, cf* dst, hipStream_t s);
void launch_gather(const ColMask& mk, const int64_t* leaf_off, const int64_t* gptr, const GatherEnt* gent, int64_t nb,
                   const cd* slots, int64_t n, int nrhs, cd* y, hipStream_t s);
// P^-1 v = alpha D^-1 alpha^T v by chunked sweeps. Block rows (elimination
// order) are grouped into chunks of consecutive rows. With L the unit lower
// block-triangular factor (L_jk = -alpha_kj^T), Linv_c the inverse of chunk
// c's diagonal part and C_c the coupling of chunk c to its folded neighbour
// range (SweepChunk):
//   forward   y_c = Linv_c r_c + (Linv_c C_c) y_range,
//             r_c = v_c + pushed terms of the entries outside the range
//   backward  z_c = Linv_c^T r'_c + (Linv_c^T C'_c) z_range,
//             r'_c = zt_c + pushed terms of the entries outside the range
// Per block row k: pos = elimination-order offset, loc = offset in its
// chunk, w = loc + b_k (forward Linv row width), wt = n_c - loc (backward
// width); row blocks of Linv (b_k x w), Linv^T (b_k x wt), Linv C (b_k x
// range width) and Linv^T C' (b_k x range width), all row-major.
template <class T>   // T: matrix storage, cd (complex128) or cf (complex64 copies)
struct SweepPlanT {
    int nb;
    int nch;
    int bmax;                  // largest block
    int64_t n;
    const int64_t* bstart;     // tree-order start of block k
    const int32_t* bsize;
    const int64_t* pos;
    const int32_t* loc;
    const int32_t* w;
    const int32_t* wt;
    const int32_t* clast;
    const int64_t* lf_off;     // Linv rows
    const int64_t* lb_off;     // Linv^T rows
    const int64_t* mf_off;     // (Linv C) rows
    const int64_t* mb_off;     // (Linv^T C^T) rows
    const T* lf;
    const T* lb;
    const T* mf;
    const T* mb;
    const int32_t* chunk_of;   // chunk of each block
    const int32_t* csize;      // points of each chunk
    // entries (k, j) outside the target chunk's folded range: pushed from their source
    // block once its chunk is final, into one slot per entry, then gathered by
    // the target block, which waits for its own count of pushed entries.
    // Forward: source k -> target j; backward: source j -> target k. Pushes are
    // grouped by source chunk (up to kPushGroup per group), nearest target
    // chunk first.
    const PushEnt* fpush;
    const int32_t* fgrp;       // per push group: first entry; entries of a group share a source chunk
    const int32_t* fgrp_n;
    const int64_t* fgptr;      // per target block: its slots (ascending source block)
    const int64_t* fgslot;
    const PushEnt* bpush;
    const int32_t* bgrp;
    const int32_t* bgrp_n;
    const int64_t* bgptr;
    const int64_t* bgslot;
    const T* alpha;
    const T* alpha_t;          // transposed copies of the dense backward push entries
    const T* dinv;
    const int64_t* dinv_off;
};
using SweepPlan = SweepPlanT<cd>;
// Work items of the non-row workgroups in ticket order: item < nb is a block
// row (phase A: r = v or D^-1 y plus its pushed slots), item >= nb the push
// group item - nb. Phase A of chunk c comes before the pushes from chunk c - 1
// (forward; mirrored backward), which come before phase A of chunk c + 1.
// Per chunk, for the row workers of one sweep direction. The folded
// neighbour range (columns of the coupling product) starts with all of the
// neighbour chunk the chain came from (c - 1 forward, c + 1 backward), whose
// values arrive last; then come the coupled source blocks of the chunks
// further away, nearest first, up to kFoldCols columns. Those are final one
// chunk earlier; their elimination-order positions are listed in a map.
struct SweepChunk {
    int32_t pc, nc;          // first elimination-order position and points of the chunk
    int32_t w2;              // width of the folded range
    int32_t l_n, l_g;        // newest neighbour chunk: its points (range columns [0, l_n)) and first position
    int32_t e_n, e_off;      // the rest (columns [l_n, w2)): points and their offset into the position map
    int32_t nblocks;         // blocks of the chunk (phase A count)
    int32_t need1, need2;    // points of chunks c -/+ 1 and c -/+ 2 (0 if absent)
    int32_t need3;           // points of chunk c -/+ 3 (0 if absent)
    int32_t pad;
};
// Per point row (indexed by elimination-order position): its slices of the
// chunk inverse (a1, width w1, first column o1 in the chunk) and of the
// folded coupling product (a2, width w2 of its chunk), and its tree-order
// position zpos (output of the backward sweep).
struct RowTask {
    int64_t a1, a2;
    int32_t w1, o1;
    int32_t zpos, pad;
};
// Persistent row workers: kRowSets sets that take turns over the chunks, each
// of kMaxChunk / 4 workgroups with one point row per wave.
constexpr int kRowWorkers = 96;
constexpr int kRowSets = 2;
// Far entries of one source chunk per push item (four waves take turns).
constexpr int kPushGroup = 16;
constexpr int kCntPad = 32;      // ints between the per-chunk sweep counters (one 128-byte line each)
struct SweepItems {
    int64_t nfwd, nbwd;      // phase A and push items of each direction
    const int32_t* fwd;
    const int32_t* bwd;
    const SweepChunk* fchunk;
    const SweepChunk* bchunk;
    const RowTask* frow;
    const RowTask* brow;
    const int32_t* femap;     // positions of the early range columns, per chunk from SweepChunk::e_off
    const int32_t* bemap;
};
// Work buffers of one apply stream: ybuf, zbuf, rbuf, rbuf2 (elimination
// order) n nrhs each; slots_f / slots_b (push results, nrhs times the slot
// totals); flags (4 nchunk + 2 nb ints: per chunk the finished phase A
// blocks and phase B rows, per target block its pushed entries, forward then
// backward; zeroed once and compared with epoch multiples); tickets (2,
// zeroed once).
struct SweepWork {
    cd* ybuf;
    cd* zbuf;
    cd* rbuf;
    cd* rbuf2;
    cd* slots_f;
    cd* slots_b;
    int* flags;
    unsigned long long* tickets;
    // flagged copies of the row results (forward y, backward z), 4 words per
    // value: word w holds 32-bit part w of the complex128 value in its low
    // half and the apply's epoch in its high half, so a reader that sees the
    // epoch in all four words has the value without a separate ready count
    unsigned long long* llf;
    unsigned long long* llb;
    // Bounded waits: a wait that has polled for wait_ticks of the constant-rate
    // device clock gives up and sets *err; every later wait of the workspace
    // sees *err and gives up at its next check, so each workgroup runs to the
    // end of the launch (on scratch data) and the host reports the timeout.
    int* err;
    long long wait_ticks;
};
constexpr int kMaxChunk = 384;   // points per chunk (bounds the row widths)
constexpr int kFoldCols = 3072;   // columns of the folded neighbour range per chunk
static_assert(kRowWorkers * 4 == kMaxChunk, "one point row per wave of the row workers");
static_assert(kFoldCols % 64 == 0 && kFoldCols >= kMaxChunk, "fold range in whole wavefront groups");
// One sweep (forward: v -> y in the work buffers; backward: D^-1 y -> z);
// the backward launch must follow the forward one of the same epoch.
// (dinv false: the backward sweep applies alpha alone, without D^-1)
void launch_sweep(bool forward, const ColMask& mk, const SweepPlan& p, const SweepItems& it, const cd* v, cd* z,
                  int nrhs, const SweepWork& w, int epoch, hipStream_t s, bool dinv = true);
void launch_sweep(bool forward, const ColMask& mk, const SweepPlanT<cf>& p, const SweepItems& it, const cd* v, cd* z,
                  int nrhs, const SweepWork& w, int epoch, hipStream_t s, bool dinv = true);
// tree order <-> the sweeps' elimination-order buffer (to_elim: tree -> elimination)
void launch_elim_move(const SweepPlan& p, const cd* src, cd* dst, int nrhs, bool to_elim, hipStream_t s);
// out = add + D^-1 in, block by block in tree order (add may be null)
void launch_block_dinv(const SweepPlan& p, const cd* in, const cd* add, cd* out, int nrhs, hipStream_t s);
int sweep_grid(int64_t nitems);
// Workgroups of the sweep kernels that can be resident at once on a device;
// the row workers spin for the whole launch, so this must exceed
// kRowSets x kRowWorkers.
int sweep_capacity(int device);
// Linv rows of every chunk from the dense in-chunk alpha blocks (intptr /
// intent: per column j the in-chunk entries (k, j), offsets into A).
void launch_linv(const SweepPlan& p, int nchunk, const int32_t* chunk_first, const int64_t* intptr,
                 const SweepEnt* intent, const cd* A, cd* lf, hipStream_t s);
// Linv^T rows from Linv rows (one workgroup per block row).
void launch_linv_transpose(const SweepPlan& p, cd* lb, hipStream_t s);
// dst (m x n row-major) = U V for low-rank blocks (U m x r column-major then V r x n row-major at src_off).
struct ExpandTask {
    int64_t src_off, dst_off;
    int32_t m, n, r, pad;
};
void launch_lr_expand(const ExpandTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s);

void launch_dots(const cd* V, int64_t ldv, int64_t vstride, int nvec, const cd* w, int64_t n, int nrhs,
                 const ColState* st, cd* partial, int nchunk, hipStream_t s);
void launch_basis_update(const cd* V, int64_t ldv, int64_t vstride, int nvec, const cd* partial, int nchunk,
                         cd* w, int64_t n, int nrhs, const ColState* st, cd* H, int64_t ldh, int mp1, int hcol,
                         bool accumulate_h, double* norm_partial, hipStream_t s);
// Hessenberg column j with its Givens rotation and stopping test, and
// v_{j+1} = w / h_{j+1,j} (ldv: column stride of v), in one launch.
void launch_givens_scale(cd* H, int64_t ldh, int m, int j, double* cs, cd* sn, cd* g, const double* norm_partial,
                         int nchunk, ColState* st, int nrhs, const cd* w, cd* vnext, int64_t ldv, int64_t n,
                         hipStream_t s);
void launch_cycle_start(const cd* r, cd* V, int64_t ldv, cd* g, int m, const double* norm_partial, int nchunk,
                        ColState* st, int64_t n, int nrhs, bool first, hipStream_t s);
void launch_col_init(ColState* st, const ColState* outer, int nrhs, double tol, int budget, hipStream_t s);
// Fresh states for the listed columns (cols, ncols entries, device) of a
// running solve whose residual partials hold ||b||^2 for them.
void launch_col_start(const double* norm_partial, int nchunk, ColState* st, int nrhs, const int* cols, int ncols,
                      double tol, int budget, int fixed, hipStream_t s);
void launch_lsq(const cd* H, int64_t ldh, int m, const cd* g, cd* y, const ColState* st, int nrhs, hipStream_t s);
void launch_combine(const cd* V, int64_t ldv, int64_t vstride, const cd* y, int m, cd* u, int64_t n, int nrhs,
                    const ColState* st, hipStream_t s);
void launch_axpy_x(cd* x, const cd* z, int64_t n, int nrhs, const ColState* st, hipStream_t s);
void launch_residual(const cd* b, const cd* zx, cd* r, int64_t n, int nrhs, double* norm_partial, int nchunk,
                     hipStream_t s);
void launch_cycle_end(const double* norm_partial, int nchunk, ColState* st, int nrhs, hipStream_t s);
void launch_col_norms(const cd* v, int64_t n, int nrhs, double* norm_partial, int nchunk, hipStream_t s);
int gmres_nchunk(int64_t n);

}  // namespace hs
