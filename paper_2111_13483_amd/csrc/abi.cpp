// C-ABI of the MI355X symmetric near-field Schur-complement preconditioner:
// handles, device memory, orchestration of the host integer phases and the
// gfx950 kernels of the build, setup and solve phases.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <thread>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "hschur.h"
#include "kernels.h"
#include "plan.h"

using hs::cd;

namespace {

thread_local std::string g_last_error;

struct Error {
    int32_t code;
    std::string msg;
};

[[noreturn]] void fail(int32_t code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(HS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int32_t set_error(const Error& e) {
    g_last_error = e.msg;
    return e.code;
}

// Device allocator bound to a context's callbacks (hipMalloc when none).
struct Mem {
    hs_alloc_fn alloc = nullptr;
    hs_free_fn freef = nullptr;
    void* user = nullptr;
    int device = 0;

    void* get(size_t bytes) {
        if (bytes == 0) bytes = 16;
        void* p = nullptr;
        if (alloc) {
            p = alloc(bytes, user);
            if (!p) fail(HS_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(HS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            }
        }
        return p;
    }
    void put(void* p) {
        if (!p) return;
        if (freef) freef(p, user);
        else (void)hipFree(p);
    }
};

// A set of device allocations released together.
struct Owned {
    Mem mem;
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    template <class T>
    T* get(size_t count) {
        T* p = static_cast<T*>(mem.get(count * sizeof(T)));
        ptrs.push_back(p);
        bytes += (int64_t)(count * sizeof(T));
        return p;
    }
    template <class T>
    T* upload(const std::vector<T>& v, hipStream_t s) {
        T* p = get<T>(std::max<size_t>(v.size(), 1));
        if (!v.empty()) hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "H2D");
        return p;
    }
    void release() {
        for (void* p : ptrs) mem.put(p);
        ptrs.clear();
        bytes = 0;
    }
    ~Owned() { release(); }
};

template <class T>
std::vector<T> download(const T* d, size_t count, hipStream_t s) {
    std::vector<T> h(count);
    if (count) {
        hip_check(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipStreamSynchronize(s), "stream sync");
    }
    return h;
}

void check_device_flag(const int* d_err, hipStream_t s) {
    int e = download(d_err, 1, s)[0];
    if (e & hs::kErrCoincident) fail(HS_EINVAL, "coincident distinct points: the kernel is singular there");
    if (e & hs::kErrSingular) fail(HS_ESINGULAR, "exactly zero pivot in a leaf-block factorisation");
    if (e & hs::kErrRankCap) fail(HS_ENUMERIC, "an ACA rank reached the rank cap without meeting the tolerance");
    if (e & hs::kErrNumeric) fail(HS_ENUMERIC, "NaN or Inf met in a leaf-block factorisation");
}

constexpr int64_t kScratchBudget = int64_t(16) << 30;  // most bytes of ACA scratch per batch

// complex64 copy of a contiguous complex128 array (count elements), owned by own
hs::cf* c64_copy(Owned& own, Owned& tmp, const cd* src, int64_t count, hipStream_t s) {
    hs::cf* dst = own.get<hs::cf>((size_t)std::max<int64_t>(count, 1));
    constexpr int64_t piece = int64_t(1) << 16;
    std::vector<hs::PtrCopy> t;
    for (int64_t o = 0; o < count; o += piece) t.push_back(hs::PtrCopy{src + o, o, std::min(piece, count - o)});
    hs::PtrCopy* d_t = tmp.upload(t, s);
    hs::launch_to_c64(d_t, (int64_t)t.size(), dst, s);
    return dst;
}

}  // namespace

// Kernel timing for measurement: while enabled, each instrumented launch is
// bracketed by a pair of events on the context's stream.
struct KernelTimer {
    bool on = false;
    int every = 1;                       // bracket every `every`-th launch of each kind
    int64_t seen[HS_KT_COUNT] = {};      // launches of each kind since timing began
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    hipEvent_t take() {
        if (pool.empty()) {
            hipEvent_t e;
            hip_check(hipEventCreate(&e), "hipEventCreate");
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    void release() {
        for (auto& r : recs) {
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    ~KernelTimer() {
        release();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// A second stream owned by the library (default priority) with a fork and a
// join event: the near-field matvec runs on it beside the far-field matvec.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void ensure() {
        if (s) return;
        hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
        hip_check(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreateWithFlags");
        hip_check(hipEventCreateWithFlags(&join, hipEventDisableTiming), "hipEventCreateWithFlags");
    }
    ~AuxStream() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (s) (void)hipStreamDestroy(s);
    }
};

// Sweeps of the preconditioner apply keep workgroups resident that wait on
// each other, so two must never run at once on a device. Applies on one
// stream are ordered by the stream; across streams (contexts, or a context
// whose stream changed) each device keeps the stream of its latest apply and
// an event: an apply on another stream waits for that event, recorded on the
// previous stream when the stream changes (or when a context moves off it),
// and after every apply once more than one stream has been seen.
struct SweepOrder {
    std::mutex mu;
    hipStream_t last = nullptr;   // stream of the latest apply not yet captured in `done`
    bool have_done = false;       // `done` holds a recorded apply that other streams must wait for
    bool multi = false;           // applies have come from more than one stream
    hipEvent_t done = nullptr;
};
SweepOrder g_sweep_order[64];

// Device scratch of the allocation-free matvec (hs_matvec_noalloc): one copy
// per device, held until the process ends. In host code `scratch` only names
// the symbol; its device address on each device comes from
// hipGetSymbolAddress (taken once per device when the first context on that
// device is created) and only that address is passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
struct ScratchAddr {
    std::mutex mu;
    void* ptr[64] = {};
};
ScratchAddr g_scratch;

struct hs_context {
    int device = 0;
    hipStream_t stream = nullptr;
    Mem mem;
    KernelTimer timer;
    AuxStream aux;
    double wait_seconds = 5.0;    // bound on a sweep's device-side waits
    double clock_khz = 0.0;       // constant-rate device clock (wall_clock64)
    rocblas_handle blas = nullptr;   // plain GEMMs of the block-GMRES comparator (created on first use)
    ~hs_context() {
        if (blas) (void)rocblas_destroy_handle(blas);
    }
};

namespace {

// Runs f (launches on s), bracketed by timing events when the timer is on.
template <class F>
void timed(hs_context* ctx, int kind, hipStream_t s, F&& f) {
    if (!ctx || !ctx->timer.on) {
        f();
        return;
    }
    if (ctx->timer.seen[kind]++ % ctx->timer.every != 0) {
        f();
        return;
    }
    KernelTimer::Rec r{kind, ctx->timer.take(), ctx->timer.take()};
    hip_check(hipEventRecord(r.a, s), "hipEventRecord");
    f();
    hip_check(hipEventRecord(r.b, s), "hipEventRecord");
    ctx->timer.recs.push_back(r);
}

}  // namespace

struct hs_plan {
    hs::Tree tree;
    hs::Partition part;
    hs::Symbolic sym;
    bool has_sym = false;
};

// Compressed blocks of one family (far field or fill-in) after ACA +
// re-compression: per block rank and device pointer to U (m x r, col-major)
// followed by V (r x n, row-major).
struct LowRankSet {
    std::vector<int> rank;          // final rank per block
    std::vector<int> rank_aca;      // rank before re-compression
    std::vector<cd*> ptr;           // device pointers (nullptr when rank 0 or not stored)
};

struct hs_hmatrix {
    Owned own;
    hs_plan plan;
    int64_t n = 0, nb = 0;
    double k = 0, h = 0;
    int rank_cap = 0;
    std::vector<int64_t> leaf_off;
    std::vector<hs::NearTask> near_tasks;
    std::vector<hs::AcaTask> far_geom;
    LowRankSet far;
    int64_t bytes_near = 0, bytes_far = 0;
    int64_t slot_total = 0;
    int64_t near_slot_end = 0;   // slots [0, near_slot_end) belong to the near blocks
    // device
    double* d_pts = nullptr;
    int64_t* d_perm = nullptr;
    int64_t* d_leaf_off = nullptr;
    hs::NearTask* d_near_tasks = nullptr;
    cd* d_near = nullptr;
    int64_t* d_near_slot = nullptr;
    // the far blocks again, largest r (m + n) first, for the matvec launch
    hs::AcaTask* d_mv_geom = nullptr;
    int* d_mv_rank = nullptr;
    int64_t n_far_wg = 0;   // matvec far tasks taken by a whole workgroup (the rest by one wave)
    cd** d_mv_ptr = nullptr;
    int64_t* d_mv_slot = nullptr;
    int* d_far_piv = nullptr;
    int64_t* d_gptr = nullptr;
    hs::GatherEnt* d_gent = nullptr;
    // complex64 copies for mixed solves (store_c64)
    bool c64 = false;
    hs::cf* d_near32 = nullptr;
    hs::cf** d_mv_ptr32 = nullptr;
    // The far field is compressed by a host thread on the H-matrix's own
    // streams while the caller goes on (a preconditioner setup reads only the
    // near field); every entry point that reads the far field joins it first.
    mutable std::thread far_thread;
    mutable std::exception_ptr far_err;
    hipStream_t far_s = nullptr;
    hipEvent_t far_start = nullptr;   // the build's uploads on the caller's stream
    AuxStream far_aux;
    void join_far() const {
        if (far_thread.joinable()) far_thread.join();
        if (far_err) std::rethrow_exception(far_err);
    }
    ~hs_hmatrix() {
        if (far_thread.joinable()) far_thread.join();
        if (far_s) (void)hipStreamDestroy(far_s);
        if (far_start) (void)hipEventDestroy(far_start);
    }
};

struct hs_precond {
    Owned own;
    const hs_hmatrix* H = nullptr;
    hs_plan plan;   // ordering + symbolic (tree/partition left empty)
    int64_t nb = 0;
    std::vector<int32_t> bsize;
    std::vector<int64_t> bstart;
    std::vector<int64_t> d_off;          // element offsets of D_k / D_k^-1
    std::vector<int64_t> a_off;          // final alpha store offsets per pattern entry
    std::vector<int> a_rank;             // -1 dense
    int64_t alpha_elems = 0, d_elems = 0;
    int64_t n_lowrank = 0, n_fill = 0, max_dk = 0;
    double flops_setup = 0, flops_fill = 0;
    double flops_factored = 0;   // HS_PC_SCHUR_LOWRANK: the elimination's flops with the replaced blocks factored
    // device
    cd* d_D = nullptr;       // final W_kk
    cd* d_dinv = nullptr;    // D_k^-1
    int64_t* d_dinv_off = nullptr;
    cd* d_alpha = nullptr;
    int64_t* d_bstart = nullptr;
    int32_t* d_bsize = nullptr;
    // chunked sweeps
    int64_t nchunk = 0, linv_elems = 0;
    int64_t fslot_total = 0, bslot_total = 0;
    hs::SweepPlan sp{};
    hs::SweepItems items{};
    int64_t alpha_t_elems = 0;
    // complex64 copies of the apply's matrices (HS_PREC_MIXED)
    bool c64 = false;
    bool block_jacobi = false;   // HS_PC_BLOCK_JACOBI: P^-1 = blockdiag(Z_kk)^-1
    // HS_PC_SCHUR_NONSYM: the left coefficients alpha'_jk, stored transposed
    // (b_k x b_j row-major, dense, pattern entries back to back)
    cd* d_alpha_left = nullptr;
    int64_t alpha_left_elems = 0;
    hs::SweepPlanT<hs::cf> sp32{};
};

namespace {

void set_device(const hs_context* ctx) { hip_check(hipSetDevice(ctx->device), "hipSetDevice"); }

// Indices 0..n-1 ordered by key descending, equal keys in index order: an
// LSD radix sort of the complemented keys, 16 bits a pass, as many passes as
// the largest key needs (a tenth of a comparison sort's time on the far
// field's 26,000 blocks, which the host sorts three times per H-matrix).
std::vector<int32_t> order_by_key_desc(const std::vector<uint64_t>& key) {
    const size_t n = key.size();
    std::vector<int32_t> a(n), b(n);
    for (size_t i = 0; i < n; ++i) a[i] = (int32_t)i;
    uint64_t mx = 0;
    for (uint64_t k : key) mx = std::max(mx, k);
    std::vector<uint32_t> cnt(size_t(1) << 16);
    for (int shift = 0; shift < 64 && (mx >> shift) != 0; shift += 16) {
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (size_t i = 0; i < n; ++i) ++cnt[((mx - key[i]) >> shift) & 0xffff];
        uint32_t sum = 0;
        for (auto& c : cnt) {
            const uint32_t t = c;
            c = sum;
            sum += t;
        }
        for (size_t i = 0; i < n; ++i) {
            const int32_t v = a[i];
            b[cnt[((mx - key[v]) >> shift) & 0xffff]++] = v;
        }
        a.swap(b);
    }
    return a;
}

// ACA + re-compression of a list of blocks in batches bounded by the scratch
// budget. Dense blocks read src (row-major m x n at src_off); otherwise the
// kernel is evaluated on the points. The final factors go into chunks owned
// by `own`; piv_log (optional) receives (i, j) per ACA step, stride 2*cap_max.
// With ax (far field), the blocks of rank above kRcWideRank are re-compressed
// by wide workgroups on the auxiliary stream beside the others.
void compress_blocks(Owned& own, hipStream_t s, std::vector<hs::AcaTask> tasks, bool dense, const double* pts,
                     double k, const cd* src, double eps, int cap_max, int* d_err, int* d_piv_log,
                     LowRankSet& out, AuxStream* ax) {
    const int64_t nt = (int64_t)tasks.size();
    out.rank.assign(nt, 0);
    out.rank_aca.assign(nt, 0);
    out.ptr.assign(nt, nullptr);
    if (nt == 0) return;
    Owned tmp;
    tmp.mem = own.mem;
    // one batch where memory allows, so the slowest blocks of the whole list
    // overlap in one launch per kernel: at most half of the free device memory
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = 0;
    }
    const int64_t budget = std::max<int64_t>(int64_t(1) << 30, std::min<int64_t>(kScratchBudget, (int64_t)(free_b / 2)));
    int64_t b0 = 0;
    while (b0 < nt) {
        // batch [b0, b1) within the scratch budget
        int64_t b1 = b0, elems = 0, flag_bytes = 0;
        while (b1 < nt) {
            hs::AcaTask& t = tasks[b1];
            t.cap = std::min(std::min(t.m, t.n), cap_max);
            int64_t e = (int64_t)(t.m + t.n) * t.cap;
            if (b1 > b0 && (elems + e) * 16 + flag_bytes > budget) break;
            t.u_off = elems;
            t.v_off = elems + (int64_t)t.m * t.cap;
            t.flag_off = flag_bytes;
            elems += e;
            flag_bytes += t.m + t.n;
            ++b1;
        }
        const int64_t nb_ = b1 - b0;
        std::vector<hs::AcaTask> bt(tasks.begin() + b0, tasks.begin() + b1);
        tmp.release();
        hs::AcaTask* d_t = tmp.upload(bt, s);
        cd* scratch = tmp.get<cd>(elems);
        uint8_t* flags = tmp.get<uint8_t>(flag_bytes);
        int* d_rank = tmp.get<int>(nb_);
        int* d_rank2 = tmp.get<int>(nb_);
        // far field: the largest blocks first (their ranks, and so their ACA
        // steps, are the largest); the fill-in blocks (leaf x leaf, similar
        // sizes) keep their order, which saves the host sort
        const int32_t* d_aorder = nullptr;
        if (!dense) {
            std::vector<uint64_t> key(nb_);
            for (int64_t i = 0; i < nb_; ++i)
                key[i] = (uint64_t)(bt[i].m + bt[i].n) * (uint64_t)std::min(bt[i].m, bt[i].n);
            d_aorder = tmp.upload(order_by_key_desc(key), s);
        }
        hs::launch_aca(dense, d_t, d_aorder, nb_, pts, k, src, scratch, flags, eps, d_rank,
                       d_piv_log ? d_piv_log + b0 * 2 * cap_max : nullptr, 2 * cap_max, d_err, s);
        hip_check(hipGetLastError(), "k_aca launch");
        std::vector<int> r = download(d_rank, nb_, s);
        std::vector<int64_t> ws_off(nb_);
        int64_t ws = 0;
        for (int64_t i = 0; i < nb_; ++i) {
            ws_off[i] = ws;
            ws += 4 * (int64_t)r[i] * r[i] + r[i];
        }
        int64_t* d_ws_off = tmp.upload(ws_off, s);
        cd* d_ws = tmp.get<cd>(ws);
        // far field: the blocks of rank above kRcWideRank (few, but the
        // slowest) on wide workgroups on the auxiliary stream, the others
        // beside them with the costliest first: QR of both factors
        // ((m + n) r^2) and the core's Jacobi sweeps (~ r^3), ties by index
        std::vector<int32_t> wide, rest;
        for (int64_t i = 0; i < nb_; ++i) {
            if (ax && r[i] > hs::kRcWideRank)
                wide.push_back((int32_t)i);
            else
                rest.push_back((int32_t)i);
        }
        const int32_t* d_wide = nullptr;
        const int32_t* d_rest = nullptr;
        // lists of small blocks only (the fill-in of leaves up to 64 points):
        // one wave per block, many resident per CU
        bool all_small = dense;
        for (int64_t i = 0; i < nb_ && all_small; ++i)
            all_small = bt[i].m <= hs::kRcSmallLen && bt[i].n <= hs::kRcSmallLen;
        const int rest_kind = all_small ? hs::kRcSmall : hs::kRcRest;
        if (!dense) {
            auto by_cost = [&](std::vector<int32_t>& list) {
                std::vector<uint64_t> key(list.size());
                for (size_t q = 0; q < list.size(); ++q) {
                    const uint64_t i = (uint64_t)list[q], rr = (uint64_t)r[i];
                    key[q] = (uint64_t)(bt[i].m + bt[i].n) * rr * rr + 10 * rr * rr * rr;
                }
                const std::vector<int32_t> o = order_by_key_desc(key);
                std::vector<int32_t> sorted(list.size());
                for (size_t q = 0; q < list.size(); ++q) sorted[q] = list[o[q]];
                list.swap(sorted);
            };
            by_cost(wide);
            by_cost(rest);
        }
        if (!wide.empty()) d_wide = tmp.upload(wide, s);
        // all blocks in index order need no list (the fill-in batches)
        if (!dense || !wide.empty()) d_rest = tmp.upload(rest, s);
        auto fork = [&] {
            if (wide.empty()) return;
            ax->ensure();
            hip_check(hipEventRecord(ax->fork, s), "hipEventRecord");
            hip_check(hipStreamWaitEvent(ax->s, ax->fork, 0), "hipStreamWaitEvent");
        };
        auto join = [&] {
            if (wide.empty()) return;
            hip_check(hipEventRecord(ax->join, ax->s), "hipEventRecord");
            hip_check(hipStreamWaitEvent(s, ax->join, 0), "hipStreamWaitEvent");
        };
        fork();
        if (!wide.empty())
            hs::launch_recompress_a(hs::kRcWide, d_t, d_wide, (int64_t)wide.size(), scratch, d_rank, d_ws, d_ws_off, eps,
                                    d_rank2, ax->s);
        hs::launch_recompress_a(rest_kind, d_t, d_rest, (int64_t)rest.size(), scratch, d_rank, d_ws, d_ws_off, eps,
                                d_rank2, s);
        hip_check(hipGetLastError(), "k_recompress_a launch");
        join();
        std::vector<int> r2 = download(d_rank2, nb_, s);
        int64_t fin = 0;
        for (int64_t i = 0; i < nb_; ++i) fin += (int64_t)r2[i] * (bt[i].m + bt[i].n);
        cd* chunk = own.get<cd>(fin);
        std::vector<cd*> dst(nb_, nullptr);
        int64_t off = 0;
        for (int64_t i = 0; i < nb_; ++i) {
            out.rank_aca[b0 + i] = r[i];
            out.rank[b0 + i] = r2[i];
            if (r2[i] > 0) {
                dst[i] = chunk + off;
                out.ptr[b0 + i] = dst[i];
                off += (int64_t)r2[i] * (bt[i].m + bt[i].n);
            }
        }
        cd** d_dst = tmp.upload(dst, s);
        fork();
        if (!wide.empty())
            hs::launch_recompress_b(hs::kRcWide, d_t, d_wide, (int64_t)wide.size(), scratch, d_rank, d_ws, d_ws_off, d_rank2,
                                    d_dst, ax->s);
        hs::launch_recompress_b(rest_kind, d_t, d_rest, (int64_t)rest.size(), scratch, d_rank, d_ws, d_ws_off, d_rank2,
                                d_dst, s);
        hip_check(hipGetLastError(), "k_recompress_b launch");
        join();
        hip_check(hipStreamSynchronize(s), "stream sync");
        b0 = b1;
    }
    tmp.release();
}

std::vector<int64_t> leaf_offsets(const hs::Tree& t) {
    std::vector<int64_t> off(t.nb() + 1);
    for (int64_t l = 0; l < t.nb(); ++l) off[l] = t.start[t.leaf_box[l]];
    off[t.nb()] = t.n;
    return off;
}

void fill_info_plan(const hs_plan& p, hs_info* info) {
    std::memset(info, 0, sizeof(*info));
    info->n = p.tree.n;
    info->nb = p.tree.nb();
    info->nbox = p.tree.nbox();
    info->n_near = p.part.n_near();
    info->n_far = p.part.n_far();
    if (p.has_sym) {
        info->n_pattern = p.sym.nnz();
        int64_t nf = 0, md = 0;
        for (int64_t e = 0; e < p.sym.nnz(); ++e) nf += p.sym.orig[e] ? 0 : 1;
        for (int64_t kk = 0; kk < p.tree.nb(); ++kk) md = std::max(md, p.sym.rowptr[kk + 1] - p.sym.rowptr[kk]);
        info->n_fill = nf;
        info->max_dk = md;
        // exact algorithmic counts of the elimination (Sec. 4): LU 8/3 b^3,
        // alpha 8 b_k^2 b_j, updates 8 b_i b_k b_j; dense alpha bytes
        const hs::Tree& t = p.tree;
        std::vector<double> b(t.nb());
        for (int64_t kk = 0; kk < t.nb(); ++kk) b[kk] = (double)t.count[t.leaf_box[p.sym.order[kk]]];
        double fl = 0, ab = 0, db = 0;
        for (int64_t kk = 0; kk < t.nb(); ++kk) {
            const double bk = b[kk];
            fl += 8.0 / 3.0 * bk * bk * bk;
            db += bk * bk * 16.0;
            double sj = 0, sj2 = 0;
            for (int64_t e = p.sym.rowptr[kk]; e < p.sym.rowptr[kk + 1]; ++e) {
                const double bj = b[p.sym.cols[e]];
                fl += 8.0 * bk * bk * bj;
                ab += bk * bj * 16.0;
                sj += bj;
                sj2 += bj * bj;
            }
            fl += 8.0 * bk * 0.5 * (sj * sj + sj2);   // sum over i <= j of b_i b_j
        }
        info->flops_setup = fl;
        info->bytes_alpha = (int64_t)ab;
        info->bytes_d = (int64_t)db;
    }
    // footprint estimate (admission before allocation): near blocks exact,
    // far factors at rank min(m, n, 32), and with a pattern three times the
    // dense scaling-coefficient bound plus the block diagonal
    const hs::Tree& t = p.tree;
    double nearb = 0, farb = 0;
    for (int64_t e = 0; e < p.part.n_near(); ++e) {
        const double bi = (double)t.count[t.leaf_box[p.part.near[2 * e]]];
        const double bj = (double)t.count[t.leaf_box[p.part.near[2 * e + 1]]];
        nearb += bi * bj * 16.0;
    }
    for (int64_t e = 0; e < p.part.n_far(); ++e) {
        const double m = (double)t.count[p.part.far[2 * e]], nn = (double)t.count[p.part.far[2 * e + 1]];
        farb += std::min(std::min(m, nn), 32.0) * (m + nn) * 16.0;
    }
    info->bytes_near = (int64_t)nearb;
    info->bytes_estimate = (int64_t)(nearb + farb + 3.0 * (double)info->bytes_alpha + (double)info->bytes_d);
}

hs::Symbolic make_symbolic(const hs_plan& p, int ordering) {
    std::vector<int64_t> order = hs::make_order(ordering, p.tree.nb(), p.part);
    return hs::symbolic(p.tree.nb(), p.part, order);
}

int32_t export_plan(const hs_plan& p, int32_t what, void* dst, int64_t cap, int64_t* needed) {
    std::vector<int64_t> v;
    const hs::Tree& t = p.tree;
    switch (what) {
        case HS_X_PERM: v = t.perm; break;
        case HS_X_LEAF_OFF: v = leaf_offsets(t); break;
        case HS_X_BOXES:
            for (int64_t b = 0; b < t.nbox(); ++b) {
                v.push_back(t.level[b]);
                v.push_back(t.start[b]);
                v.push_back(t.count[b]);
                for (int a = 0; a < 3; ++a) v.push_back(t.anchor[3 * b + a]);
                v.push_back(t.leaf_id[b]);
            }
            break;
        case HS_X_NEAR: v = p.part.near; break;
        case HS_X_FAR: v = p.part.far; break;
        case HS_X_ORDER:
        case HS_X_ROWPTR:
        case HS_X_COLS:
        case HS_X_ORIG:
            if (!p.has_sym) fail(HS_EINVAL, "the plan has no ordering");
            v = what == HS_X_ORDER ? p.sym.order
              : what == HS_X_ROWPTR ? p.sym.rowptr
              : what == HS_X_COLS ? p.sym.cols : p.sym.orig;
            break;
        default: fail(HS_EINVAL, "unknown export code");
    }
    const int64_t bytes = (int64_t)(v.size() * sizeof(int64_t));
    if (needed) *needed = bytes;
    if (!dst) return HS_OK;
    if (cap < bytes) fail(HS_EINVAL, "export buffer too small");
    if (bytes) std::memcpy(dst, v.data(), bytes);
    return HS_OK;
}

int32_t copy_out(const void* src_dev, int64_t bytes, void* dst, int64_t cap, int64_t* needed, hipStream_t s) {
    if (needed) *needed = bytes;
    if (!dst) return HS_OK;
    if (cap < bytes) fail(HS_EINVAL, "export buffer too small");
    if (bytes) {
        hip_check(hipMemcpyAsync(dst, src_dev, bytes, hipMemcpyDeviceToHost, s), "D2H export");
        hip_check(hipStreamSynchronize(s), "stream sync");
    }
    return HS_OK;
}

template <class T>
int32_t copy_host(const std::vector<T>& v, void* dst, int64_t cap, int64_t* needed) {
    const int64_t bytes = (int64_t)(v.size() * sizeof(T));
    if (needed) *needed = bytes;
    if (!dst) return HS_OK;
    if (cap < bytes) fail(HS_EINVAL, "export buffer too small");
    if (bytes) std::memcpy(dst, v.data(), bytes);
    return HS_OK;
}

// ---- operator applications on tree-order vectors ------------------------------

struct MatvecWs {
    cd* slots = nullptr;
};

// mk selects the columns computed (all for the public entry points)
// Near and far matvec write disjoint slot ranges and only read x, so the near
// part runs on the auxiliary stream beside the far part; the gather waits for
// both. The fork follows all earlier work on s. (The wave-sized far blocks on
// a third stream made the c2 solve 2% slower: the three kernels then compete
// for the same CUs; on this stream after the near blocks, 1.5% slower.)
void matvec_tree(hs_context* ctx, const hs_hmatrix* H, const cd* x, cd* y, int nrhs, cd* slots, hipStream_t s,
                 const hs::ColMask& mk) {
    AuxStream& ax = ctx->aux;
    ax.ensure();
    hip_check(hipEventRecord(ax.fork, s), "hipEventRecord");
    hip_check(hipStreamWaitEvent(ax.s, ax.fork, 0), "hipStreamWaitEvent");
    timed(ctx, HS_KT_NEAR_MV, ax.s, [&] {
        hs::launch_near_mv(mk, H->d_near_tasks, H->d_near_slot, (int64_t)H->near_tasks.size(), H->d_near, x, H->n,
                           nrhs, slots, ax.s);
    });
    timed(ctx, HS_KT_FAR_MV, s, [&] {
        hs::launch_far_mv(mk, H->d_mv_geom, H->d_mv_rank, H->d_mv_ptr, H->d_mv_slot, H->n_far_wg,
                          (int64_t)H->far_geom.size(), x, H->n, nrhs, slots, s);
    });
    hip_check(hipEventRecord(ax.join, ax.s), "hipEventRecord");
    hip_check(hipStreamWaitEvent(s, ax.join, 0), "hipStreamWaitEvent");
    hs::launch_gather(mk, H->d_leaf_off, H->d_gptr, H->d_gent, H->nb, slots, H->n, nrhs, y, s);
}

// A sweep direction's counters advance with its own epoch, so forward and
// backward sweeps may also run alone (the transformed system applies
// alpha^T and alpha separately).
struct SweepWs {
    hs::SweepWork w{};
    int epoch_f = 0, epoch_b = 0;
};

SweepOrder& sweep_order(int device) {
    if (device < 0 || device >= 64) fail(HS_EINVAL, "device index beyond the library's table");
    return g_sweep_order[device];
}

// Called before the sweeps of an apply on stream s (see SweepOrder).
void sweeps_begin(int device, hipStream_t s) {
    SweepOrder& o = sweep_order(device);
    std::lock_guard<std::mutex> lk(o.mu);
    if (o.last != nullptr && o.last != s) {
        if (!o.done) hip_check(hipEventCreateWithFlags(&o.done, hipEventDisableTiming), "hipEventCreateWithFlags");
        hip_check(hipEventRecord(o.done, o.last), "hipEventRecord");
        o.have_done = true;
        o.multi = true;
        o.last = nullptr;
    }
    if (o.last == nullptr && o.have_done) hip_check(hipStreamWaitEvent(s, o.done, 0), "hipStreamWaitEvent");
    o.last = s;
}

// Called after the sweeps of an apply on stream s.
void sweeps_end(int device, hipStream_t s) {
    SweepOrder& o = sweep_order(device);
    std::lock_guard<std::mutex> lk(o.mu);
    if (!o.multi) return;
    hip_check(hipEventRecord(o.done, s), "hipEventRecord");
    o.have_done = true;
}

// A context moves off stream s (new stream or destruction): capture its
// latest apply while s is still valid.
void sweeps_release(int device, hipStream_t s) {
    SweepOrder& o = sweep_order(device);
    std::lock_guard<std::mutex> lk(o.mu);
    if (o.last != s || s == nullptr) return;
    if (!o.done && hipEventCreateWithFlags(&o.done, hipEventDisableTiming) != hipSuccess) return;
    if (hipEventRecord(o.done, s) == hipSuccess) o.have_done = true;
    o.multi = true;
    o.last = nullptr;
}

void apply_tree(hs_context* ctx, const hs_precond* P, const cd* v, cd* z, int nrhs, SweepWs& ws, hipStream_t s,
                const hs::ColMask& mk) {
    if (P->block_jacobi) {
        hs::launch_block_dinv(P->sp, v, nullptr, z, nrhs, s);
        return;
    }
    ws.epoch_f += 1;
    ws.epoch_b += 1;
    sweeps_begin(ctx->device, s);
    timed(ctx, HS_KT_SWEEP_FWD, s,
          [&] { hs::launch_sweep(true, mk, P->sp, P->items, v, z, nrhs, ws.w, ws.epoch_f, s); });
    timed(ctx, HS_KT_SWEEP_BWD, s,
          [&] { hs::launch_sweep(false, mk, P->sp, P->items, v, z, nrhs, ws.w, ws.epoch_b, s); });
    sweeps_end(ctx->device, s);
}

// alpha^T v (forward sweep alone; tree order in and out; tmp: elimination-order scratch unused)
void alpha_t_tree(hs_context* ctx, const hs_precond* P, const cd* v, cd* out, int nrhs, SweepWs& ws, hipStream_t s,
                  const hs::ColMask& mk) {
    ws.epoch_f += 1;
    sweeps_begin(ctx->device, s);
    timed(ctx, HS_KT_SWEEP_FWD, s,
          [&] { hs::launch_sweep(true, mk, P->sp, P->items, v, out, nrhs, ws.w, ws.epoch_f, s); });
    sweeps_end(ctx->device, s);
    hs::launch_elim_move(P->sp, ws.w.ybuf, out, nrhs, false, s);
}

// alpha u (backward sweep without D^-1; tree order in and out)
void alpha_tree(hs_context* ctx, const hs_precond* P, const cd* u, cd* out, int nrhs, SweepWs& ws, hipStream_t s,
                const hs::ColMask& mk) {
    hs::launch_elim_move(P->sp, u, ws.w.ybuf, nrhs, true, s);
    ws.epoch_b += 1;
    sweeps_begin(ctx->device, s);
    timed(ctx, HS_KT_SWEEP_BWD, s,
          [&] { hs::launch_sweep(false, mk, P->sp, P->items, u, out, nrhs, ws.w, ws.epoch_b, s, false); });
    sweeps_end(ctx->device, s);
}

// The sweeps' error flag (bounded waits) of a workspace, read after a
// synchronisation point the caller already pays for.
void check_sweep_flag(const SweepWs& ws, hipStream_t s) {
    if (!ws.w.err) return;
    if (download(ws.w.err, 1, s)[0] != 0)
        fail(HS_ETIMEOUT, "a device-side wait of the preconditioner sweeps exceeded the context's wait limit");
}

const hs::ColMask kAllCols{nullptr, 0, 0};

SweepWs make_sweep_ws(Owned& o, const hs_precond* P, int nrhs, hipStream_t s, const hs_context* ctx) {
    SweepWs sw;
    sw.w.err = o.get<int>(1);
    hip_check(hipMemsetAsync(sw.w.err, 0, sizeof(int), s), "memset err");
    const double ticks = ctx->wait_seconds * ctx->clock_khz * 1e3;
    sw.w.wait_ticks = ticks < 9e18 ? (long long)ticks : (long long)9e18;
    const size_t nn = (size_t)P->H->n * nrhs;
    sw.w.ybuf = o.get<cd>(nn);
    sw.w.zbuf = o.get<cd>(nn);
    sw.w.rbuf = o.get<cd>(nn);
    sw.w.rbuf2 = o.get<cd>(nn);
    sw.w.slots_f = o.get<cd>((size_t)std::max<int64_t>(P->fslot_total, 1) * nrhs);
    sw.w.slots_b = o.get<cd>((size_t)std::max<int64_t>(P->bslot_total, 1) * nrhs);
    const size_t nflags = (size_t)4 * hs::kCntPad * P->nchunk + (size_t)2 * P->nb;
    sw.w.flags = o.get<int>(nflags);
    sw.w.tickets = o.get<unsigned long long>(2);
    hip_check(hipMemsetAsync(sw.w.flags, 0, sizeof(int) * nflags, s), "memset flags");
    hip_check(hipMemsetAsync(sw.w.tickets, 0, sizeof(unsigned long long) * 2, s), "memset tickets");
    // epochs start at 1 for each workspace: clear the flagged copies so no
    // stale word of an earlier workspace carries a matching epoch
    sw.w.llf = o.get<unsigned long long>(4 * nn);
    sw.w.llb = o.get<unsigned long long>(4 * nn);
    hip_check(hipMemsetAsync(sw.w.llf, 0, sizeof(unsigned long long) * 4 * nn, s), "memset llf");
    hip_check(hipMemsetAsync(sw.w.llb, 0, sizeof(unsigned long long) * 4 * nn, s), "memset llb");
    return sw;
}

}  // namespace

// =============================================================================== C-ABI

namespace {

// The far field of an H-matrix: ACA + re-compression of every far block,
// the matvec's slot layout, gather lists and launch order, and the complex64
// copies when asked for; on the H-matrix's own stream H->far_s (run by the
// build's far-field host thread).
void build_far(hs_hmatrix* H, double k, double aca_tol, int cap, bool store_c64, int* d_err) {
    hipStream_t s = H->far_s;
    Owned& o = H->own;
    const hs::Tree& t = H->plan.tree;
    const hs::Partition& p = H->plan.part;
    // matvec slots and per-leaf gather lists (fixed summation order): they
    // depend on the partition only, so a host thread builds them while
    // the far field is compressed on the GPU
    std::vector<int64_t> near_slot(H->near_tasks.size()), far_slot(H->far_geom.size());
    std::vector<int64_t> gptr(t.nb() + 1, 0);
    std::vector<hs::GatherEnt> gent;
    int64_t near_slot_end = 0, slot_total = 0;
    std::exception_ptr gl_err;
    std::thread gl_thread([&] {
        try {
            std::vector<std::vector<hs::GatherEnt>> lists(t.nb());
            int64_t slot = 0;
            for (int64_t e = 0; e < p.n_near(); ++e) {
                const int64_t i = p.near[2 * e], j = p.near[2 * e + 1];
                const hs::NearTask& nt = H->near_tasks[e];
                near_slot[e] = slot;
                lists[i].push_back(hs::GatherEnt{slot, nt.m, 0});
                if (i != j) lists[j].push_back(hs::GatherEnt{slot + nt.m, nt.n, 0});
                slot += nt.m + (i != j ? nt.n : 0);
            }
            near_slot_end = slot;
            // leaves of a box: leaf starts are sorted, boxes are contiguous point ranges
            auto leaves_of = [&](int64_t b, int64_t& l0, int64_t& l1) {
                const int64_t s0 = t.start[b], s1 = t.start[b] + t.count[b];
                l0 = std::lower_bound(H->leaf_off.begin(), H->leaf_off.end() - 1, s0) - H->leaf_off.begin();
                l1 = std::lower_bound(H->leaf_off.begin(), H->leaf_off.end() - 1, s1) - H->leaf_off.begin();
            };
            for (int64_t e = 0; e < p.n_far(); ++e) {
                const hs::AcaTask& g = H->far_geom[e];
                far_slot[e] = slot;
                int64_t l0, l1;
                leaves_of(p.far[2 * e], l0, l1);
                for (int64_t l = l0; l < l1; ++l)
                    lists[l].push_back(hs::GatherEnt{slot, g.m, (int32_t)(H->leaf_off[l] - g.t0)});
                leaves_of(p.far[2 * e + 1], l0, l1);
                for (int64_t l = l0; l < l1; ++l)
                    lists[l].push_back(hs::GatherEnt{slot + g.m, g.n, (int32_t)(H->leaf_off[l] - g.s0)});
                slot += g.m + g.n;
            }
            slot_total = slot;
            for (int64_t l = 0; l < t.nb(); ++l) {
                gent.insert(gent.end(), lists[l].begin(), lists[l].end());
                gptr[l + 1] = (int64_t)gent.size();
            }
        } catch (...) {
            gl_err = std::current_exception();
        }
    });
    struct Joiner {
        std::thread& th;
        ~Joiner() {
            if (th.joinable()) th.join();
        }
    } gl_join{gl_thread};
    compress_blocks(o, s, H->far_geom, false, H->d_pts, k, nullptr, aca_tol, cap, d_err, H->d_far_piv, H->far,
                    &H->far_aux);
    gl_thread.join();
    if (gl_err) std::rethrow_exception(gl_err);
    H->near_slot_end = near_slot_end;
    H->slot_total = slot_total;
    check_device_flag(d_err, s);
    int64_t fb = 0;
    for (size_t b = 0; b < H->far_geom.size(); ++b) {
        H->far_geom[b].cap = cap;
        fb += (int64_t)H->far.rank[b] * (H->far_geom[b].m + H->far_geom[b].n);
    }
    H->bytes_far = fb * 16;
    H->d_near_slot = o.upload(near_slot, s);
    {
        // the matvec takes the workgroup blocks largest first so the long
        // ones do not trail the launch, then the blocks small enough for
        // one wave (at most 64 x 64 points, rank <= kFarWaveRank)
        const int64_t nf = p.n_far();
        auto cost = [&](int64_t e) {
            return (uint64_t)H->far.rank[e] * (uint64_t)(H->far_geom[e].m + H->far_geom[e].n);
        };
        auto wave = [&](int64_t e) {
            return H->far_geom[e].m <= 64 && H->far_geom[e].n <= 64 && H->far.rank[e] <= hs::kFarWaveRank;
        };
        // workgroup blocks (bit 62 set) before wave blocks, each by cost
        std::vector<uint64_t> key(nf);
        for (int64_t e = 0; e < nf; ++e) key[e] = (wave(e) ? 0 : uint64_t(1) << 62) | cost(e);
        const std::vector<int32_t> ord = order_by_key_desc(key);
        H->n_far_wg = 0;
        for (int64_t e = 0; e < nf; ++e) H->n_far_wg += wave(e) ? 0 : 1;
        std::vector<hs::AcaTask> mg(nf);
        std::vector<int> mr(nf);
        std::vector<cd*> mp(nf);
        std::vector<int64_t> ms(nf);
        for (int64_t q = 0; q < nf; ++q) {
            mg[q] = H->far_geom[ord[q]];
            mr[q] = H->far.rank[ord[q]];
            mp[q] = H->far.ptr[ord[q]];
            ms[q] = far_slot[ord[q]];
        }
        H->d_mv_geom = o.upload(mg, s);
        H->d_mv_rank = o.upload(mr, s);
        H->d_mv_ptr = o.upload(mp, s);
        H->d_mv_slot = o.upload(ms, s);
        if (store_c64) {
            Owned tmp;
            tmp.mem = o.mem;
            H->d_near32 = c64_copy(o, tmp, H->d_near, H->bytes_near / 16, s);
            int64_t tot = 0;
            for (int64_t q = 0; q < nf; ++q) tot += (int64_t)mr[q] * (mg[q].m + mg[q].n);
            hs::cf* base = o.get<hs::cf>((size_t)std::max<int64_t>(tot, 1));
            std::vector<hs::PtrCopy> t;
            std::vector<hs::cf*> mp32(nf, nullptr);
            int64_t off = 0;
            for (int64_t q = 0; q < nf; ++q) {
                const int64_t cnt = (int64_t)mr[q] * (mg[q].m + mg[q].n);
                mp32[q] = base + off;
                if (cnt) t.push_back(hs::PtrCopy{mp[q], off, cnt});
                off += cnt;
            }
            hs::PtrCopy* d_t = tmp.upload(t, s);
            hs::launch_to_c64(d_t, (int64_t)t.size(), base, s);
            H->d_mv_ptr32 = o.upload(mp32, s);
            hip_check(hipStreamSynchronize(s), "stream sync");
            H->c64 = true;
        }
    }
    H->d_gptr = o.upload(gptr, s);
    H->d_gent = o.upload(gent, s);
    hip_check(hipStreamSynchronize(s), "stream sync");
}

}  // namespace

extern "C" {

const char* hs_status_string(int32_t st) {
    switch (st) {
        case HS_OK: return "ok";
        case HS_NOT_CONVERGED: return "not converged";
        case HS_EINVAL: return "invalid argument";
        case HS_ENOMEM: return "out of memory";
        case HS_ENODEVICE: return "no usable gfx950 device";
        case HS_EHIP: return "HIP runtime error";
        case HS_ESINGULAR: return "singular leaf block";
        case HS_ENUMERIC: return "numerical failure";
        case HS_ETIMEOUT: return "device wait timed out";
        default: return "unknown status";
    }
}

const char* hs_last_error(void) { return g_last_error.c_str(); }

int32_t hs_context_create(hs_context** out, int32_t device, void* hip_stream, hs_alloc_fn alloc, hs_free_fn free_fn,
                          void* user) {
    try {
        if (!out) fail(HS_EINVAL, "out is NULL");
        *out = nullptr;
        if ((alloc == nullptr) != (free_fn == nullptr)) fail(HS_EINVAL, "alloc and free must be given together");
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
            (void)hipGetLastError();
            fail(HS_ENODEVICE, "no HIP device present");
        }
        if (device < 0 || device >= count) fail(HS_ENODEVICE, "device index out of range");
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            fail(HS_ENODEVICE, std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950");
        int khz = 0;
        hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device), "hipDeviceGetAttribute");
        if (khz <= 0) fail(HS_ENODEVICE, "the device reports no constant-rate clock");
        if (device >= 64) fail(HS_ENODEVICE, "device index beyond the library's table (64)");
        {
            std::lock_guard<std::mutex> lk(g_scratch.mu);
            if (!g_scratch.ptr[device]) {
                hip_check(hipSetDevice(device), "hipSetDevice");
                void* p = nullptr;
                hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
                g_scratch.ptr[device] = p;
            }
        }
        auto* c = new hs_context;
        c->clock_khz = khz;
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->mem.alloc = alloc;
        c->mem.freef = free_fn;
        c->mem.user = user;
        c->mem.device = device;
        *out = c;
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_context_set_stream(hs_context* ctx, void* hip_stream) {
    if (!ctx) { g_last_error = "ctx is NULL"; return HS_EINVAL; }
    if (static_cast<hipStream_t>(hip_stream) != ctx->stream) {
        (void)hipSetDevice(ctx->device);
        sweeps_release(ctx->device, ctx->stream);
    }
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return HS_OK;
}

int32_t hs_context_set_wait_limit(hs_context* ctx, double seconds) {
    if (!ctx) { g_last_error = "ctx is NULL"; return HS_EINVAL; }
    if (!(seconds >= 0.0)) { g_last_error = "the wait limit must be >= 0"; return HS_EINVAL; }
    ctx->wait_seconds = seconds;
    return HS_OK;
}

void hs_context_destroy(hs_context* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    sweeps_release(ctx->device, ctx->stream);
    delete ctx;
}

int32_t hs_timing_begin_every(hs_context* ctx, int32_t every) {
    try {
        if (!ctx) fail(HS_EINVAL, "ctx is NULL");
        if (every < 1) fail(HS_EINVAL, "every must be >= 1");
        set_device(ctx);
        ctx->timer.release();
        ctx->timer.every = every;
        for (int64_t& c : ctx->timer.seen) c = 0;
        ctx->timer.on = true;
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_timing_begin(hs_context* ctx) { return hs_timing_begin_every(ctx, 1); }

int32_t hs_timing_end(hs_context* ctx, hs_kernel_times* out) {
    try {
        if (!ctx || !out) fail(HS_EINVAL, "NULL argument");
        set_device(ctx);
        std::memset(out, 0, sizeof(*out));
        ctx->timer.on = false;
        for (int k = 0; k < HS_KT_COUNT; ++k) out->all_launches[k] = ctx->timer.seen[k];
        hip_check(hipStreamSynchronize(ctx->stream), "stream sync");
        for (const auto& r : ctx->timer.recs) {
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
            out->launches[r.kind] += 1;
            out->total_ms[r.kind] += ms;
        }
        ctx->timer.release();
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

// ---- plan -----------------------------------------------------------------------

int32_t hs_plan_create(const double* pts, int64_t n, int32_t leaf_max, int32_t ordering, hs_plan** out) {
    try {
        if (!out) fail(HS_EINVAL, "out is NULL");
        *out = nullptr;
        if (!pts) fail(HS_EINVAL, "points is NULL");
        if (n < 1) fail(HS_EINVAL, "n must be >= 1");
        if (leaf_max < 1) fail(HS_EINVAL, "leaf_max must be >= 1");
        if (ordering < 0 || ordering > 4) fail(HS_EINVAL, "unknown ordering");
        auto p = std::make_unique<hs_plan>();
        try {
            p->tree = hs::build_tree(pts, n, leaf_max);
        } catch (const std::invalid_argument& e) {
            fail(HS_EINVAL, e.what());
        }
        p->part = hs::build_partition(p->tree);
        p->sym = make_symbolic(*p, ordering);
        p->has_sym = true;
        *out = p.release();
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return HS_ENOMEM;
    }
}

int32_t hs_plan_query(const hs_plan* plan, hs_info* info) {
    if (!plan || !info) { g_last_error = "NULL argument"; return HS_EINVAL; }
    fill_info_plan(*plan, info);
    return HS_OK;
}

void hs_plan_destroy(hs_plan* plan) { delete plan; }

int32_t hs_plan_export(const hs_plan* plan, int32_t what, void* dst, int64_t cap, int64_t* needed) {
    try {
        if (!plan) fail(HS_EINVAL, "plan is NULL");
        return export_plan(*plan, what, dst, cap, needed);
    } catch (const Error& e) {
        return set_error(e);
    }
}

// ---- H-matrix build ----------------------------------------------------------------

int32_t hs_h_build(hs_context* ctx, const double* points_xyz, int64_t n, double k, double self_h,
                   const hs_build_opts* opts, hs_hmatrix** out) {
    try {
        if (!out) fail(HS_EINVAL, "out is NULL");
        *out = nullptr;
        if (!ctx || !points_xyz || !opts) fail(HS_EINVAL, "NULL argument");
        if (n < 1) fail(HS_EINVAL, "n must be >= 1");
        if (!(k >= 0.0) || !std::isfinite(k)) fail(HS_EINVAL, "k must be finite and >= 0");
        if (!(self_h > 0.0) || !std::isfinite(self_h)) fail(HS_EINVAL, "self_h must be > 0");
        if (opts->leaf_max < 1 || opts->leaf_max > hs::kMaxLeaf)
            fail(HS_EINVAL, "leaf_max must be in [1, " + std::to_string(hs::kMaxLeaf) + "]");
        if (!(opts->aca_tol > 0.0)) fail(HS_EINVAL, "aca_tol must be > 0");
        const int cap = opts->rank_cap > 0 ? opts->rank_cap : hs::kMaxRankCap;
        if (cap > hs::kMaxRankCap) fail(HS_EINVAL, "rank_cap above " + std::to_string(hs::kMaxRankCap));
        set_device(ctx);
        hipStream_t s = ctx->stream;
        std::vector<double> hp = download(points_xyz, (size_t)(3 * n), s);
        auto H = std::make_unique<hs_hmatrix>();
        H->own.mem = ctx->mem;
        try {
            H->plan.tree = hs::build_tree(hp.data(), n, opts->leaf_max);
        } catch (const std::invalid_argument& e) {
            fail(HS_EINVAL, e.what());
        }
        const hs::Tree& t = H->plan.tree;
        for (int64_t l = 0; l < t.nb(); ++l)
            if (t.count[t.leaf_box[l]] > hs::kMaxLeaf) fail(HS_EINVAL, "a leaf holds more points than the kernels take");
        // coincident points share a Morton key: compare within runs of equal keys
        for (int64_t i = 0; i < n;) {
            int64_t j = i + 1;
            while (j < n && t.keys[j] == t.keys[i]) ++j;
            for (int64_t a = i; a < j; ++a)
                for (int64_t b = a + 1; b < j; ++b) {
                    const double* pa = &hp[3 * t.perm[a]];
                    const double* pb = &hp[3 * t.perm[b]];
                    if (pa[0] == pb[0] && pa[1] == pb[1] && pa[2] == pb[2])
                        fail(HS_EINVAL, "coincident distinct points (duplicate input point)");
                }
            i = j;
        }
        H->plan.part = hs::build_partition(t);
        const hs::Partition& p = H->plan.part;
        H->n = n;
        H->nb = t.nb();
        H->k = k;
        H->h = self_h;
        H->rank_cap = cap;
        H->leaf_off = leaf_offsets(t);
        std::vector<double> pts_tree(3 * n);
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) pts_tree[3 * i + a] = hp[3 * t.perm[i] + a];
        Owned& o = H->own;
        H->d_pts = o.upload(pts_tree, s);
        H->d_perm = o.upload(t.perm, s);
        H->d_leaf_off = o.upload(H->leaf_off, s);
        int* d_err = o.get<int>(1);
        hip_check(hipMemsetAsync(d_err, 0, sizeof(int), s), "memset");
        // near field
        int64_t off = 0;
        for (int64_t e = 0; e < p.n_near(); ++e) {
            const int64_t i = p.near[2 * e], j = p.near[2 * e + 1];
            hs::NearTask nt;
            nt.off = off;
            nt.i0 = (int32_t)H->leaf_off[i];
            nt.m = (int32_t)(H->leaf_off[i + 1] - H->leaf_off[i]);
            nt.j0 = (int32_t)H->leaf_off[j];
            nt.n = (int32_t)(H->leaf_off[j + 1] - H->leaf_off[j]);
            off += (int64_t)nt.m * nt.n;
            H->near_tasks.push_back(nt);
        }
        H->bytes_near = off * 16;
        H->d_near = o.get<cd>(off);
        H->d_near_tasks = o.upload(H->near_tasks, s);
        hs::launch_near_assemble(H->d_near_tasks, (int64_t)H->near_tasks.size(), H->d_pts, k, self_h, H->d_near, d_err, s);
        hip_check(hipGetLastError(), "k_near_assemble launch");
        // far field
        for (int64_t e = 0; e < p.n_far(); ++e) {
            const int64_t bt = p.far[2 * e], bs = p.far[2 * e + 1];
            hs::AcaTask a{};
            a.src_off = 0;
            a.t0 = (int32_t)t.start[bt];
            a.m = (int32_t)t.count[bt];
            a.s0 = (int32_t)t.start[bs];
            a.n = (int32_t)t.count[bs];
            H->far_geom.push_back(a);
        }
        H->d_far_piv = o.get<int>((size_t)std::max<int64_t>(p.n_far(), 1) * 2 * cap);
        hip_check(hipMemsetAsync(H->d_far_piv, 0xff, sizeof(int) * std::max<int64_t>(p.n_far(), 1) * 2 * cap, s), "memset");
        // the far field on the H-matrix's own streams, after this stream's
        // uploads; a host thread runs it while the caller goes on
        int* d_err_far = o.get<int>(1);
        hip_check(hipMemsetAsync(d_err_far, 0, sizeof(int), s), "memset");
        hip_check(hipStreamCreateWithFlags(&H->far_s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
        hip_check(hipEventCreateWithFlags(&H->far_start, hipEventDisableTiming), "hipEventCreateWithFlags");
        hip_check(hipEventRecord(H->far_start, s), "hipEventRecord");
        hip_check(hipStreamWaitEvent(H->far_s, H->far_start, 0), "hipStreamWaitEvent");
        {
            hs_hmatrix* Hp = H.get();
            const int dev = ctx->device;
            const double aca_tol = opts->aca_tol;
            const bool store_c64 = opts->store_c64 != 0;
            Hp->far_thread = std::thread([Hp, dev, k, aca_tol, cap, store_c64, d_err_far] {
                try {
                    hip_check(hipSetDevice(dev), "hipSetDevice");
                    build_far(Hp, k, aca_tol, cap, store_c64, d_err_far);
                } catch (...) {
                    Hp->far_err = std::current_exception();
                }
            });
        }
        check_device_flag(d_err, s);   // the near field's (synchronises this stream)
        *out = H.release();
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return HS_ENOMEM;
    }
}

int32_t hs_query_hmatrix(const hs_hmatrix* H, hs_info* info) {
    if (!H || !info) { g_last_error = "NULL argument"; return HS_EINVAL; }
    try {
        H->join_far();
    } catch (const Error& e) {
        return set_error(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return HS_ENOMEM;
    }
    fill_info_plan(H->plan, info);
    info->bytes_near = H->bytes_near;
    info->bytes_far = H->bytes_far;
    int64_t mr = 0;
    for (int r : H->far.rank) mr = std::max<int64_t>(mr, r);
    info->max_rank = mr;
    info->bytes_device = H->own.bytes;
    return HS_OK;
}

void hs_hmatrix_destroy(hs_hmatrix* H) { delete H; }

int32_t hs_hmatrix_export(const hs_hmatrix* H, int32_t what, void* dst, int64_t cap, int64_t* needed) {
    try {
        if (!H) fail(HS_EINVAL, "H is NULL");
        if (what >= HS_X_PERM && what <= HS_X_FAR) return export_plan(H->plan, what, dst, cap, needed);
        H->join_far();
        hip_check(hipSetDevice(H->own.mem.device), "hipSetDevice");
        hipStream_t s = nullptr;
        hip_check(hipDeviceSynchronize(), "device sync");
        switch (what) {
            case HS_H_NEAR_OFF: {
                std::vector<int64_t> v;
                for (auto& t : H->near_tasks) v.push_back(t.off);
                v.push_back(H->bytes_near / 16);
                return copy_host(v, dst, cap, needed);
            }
            case HS_H_NEAR_DATA: return copy_out(H->d_near, H->bytes_near, dst, cap, needed, s);
            case HS_H_FAR_RANK: {
                std::vector<int64_t> v(H->far.rank.begin(), H->far.rank.end());
                return copy_host(v, dst, cap, needed);
            }
            case HS_H_FAR_OFF: {
                std::vector<int64_t> v(1, 0);
                for (size_t b = 0; b < H->far_geom.size(); ++b)
                    v.push_back(v.back() + (int64_t)H->far.rank[b] * (H->far_geom[b].m + H->far_geom[b].n));
                return copy_host(v, dst, cap, needed);
            }
            case HS_H_FAR_UV: {
                int64_t tot = 0;
                for (size_t b = 0; b < H->far_geom.size(); ++b)
                    tot += (int64_t)H->far.rank[b] * (H->far_geom[b].m + H->far_geom[b].n);
                if (needed) *needed = tot * 16;
                if (!dst) return HS_OK;
                if (cap < tot * 16) fail(HS_EINVAL, "export buffer too small");
                char* d = static_cast<char*>(dst);
                for (size_t b = 0; b < H->far_geom.size(); ++b) {
                    const int64_t e = (int64_t)H->far.rank[b] * (H->far_geom[b].m + H->far_geom[b].n) * 16;
                    if (e) hip_check(hipMemcpy(d, H->far.ptr[b], e, hipMemcpyDeviceToHost), "D2H");
                    d += e;
                }
                return HS_OK;
            }
            case HS_H_FAR_PIV: {
                const int64_t cnt = (int64_t)H->far_geom.size() * 2 * H->rank_cap;
                std::vector<int> raw = download(H->d_far_piv, (size_t)cnt, s);
                std::vector<int64_t> v(raw.begin(), raw.end());
                return copy_host(v, dst, cap, needed);
            }
            default: fail(HS_EINVAL, "unknown export code");
        }
    } catch (const Error& e) {
        return set_error(e);
    }
}

}  // extern "C"

namespace {

// One preconditioner setup, in phases so that the elimination steps of several
// geometries can share launches (hs_precond_setup_many).
// The Schur tiles of one step: (ti, tj) covers panel rows kSchurRows ti ..
// and columns 64 tj .. of the product W_kS^T alpha_kS and is listed when it
// holds an element with block(row) <= block(column), i.e. when the block of
// its first row is <= the block of its last column (pc: panel column starts
// of the step's blocks, m columns).
void schur_tile_list(const int32_t* pc, int32_t m, std::vector<std::pair<int16_t, int16_t>>& out) {
    const int32_t nr = (m + hs::kSchurRows - 1) / hs::kSchurRows, nc = (m + 63) / 64;
    std::vector<int32_t> afirst(nr), alast(nc);
    int32_t a = 0;
    for (int32_t t = 0; t < nr; ++t) {
        while (pc[a + 1] <= hs::kSchurRows * t) ++a;
        afirst[t] = a;
    }
    a = 0;
    for (int32_t t = 0; t < nc; ++t) {
        const int32_t g = std::min(64 * t + 63, m - 1);
        while (pc[a + 1] <= g) ++a;
        alast[t] = a;
    }
    for (int32_t ti = 0; ti < nr; ++ti)
        for (int32_t tj = 0; tj < nc; ++tj)
            if (afirst[ti] <= alast[tj]) out.emplace_back((int16_t)ti, (int16_t)tj);
}

struct SetupJob {
    hs_context* ctx = nullptr;
    const hs_hmatrix* H = nullptr;
    const hs_precond_opts* opts = nullptr;
    hipStream_t s = nullptr;
    int32_t chunk_lim = 0, fold_cols = 0;
    std::unique_ptr<hs_precond> P;
    int64_t nb = 0, nnz = 0;
    std::vector<int64_t> row_of, wd_off, w_off, ad_off;
    int64_t wtot = 0, atot = 0, dtot = 0;
    Owned tmp;
    cd* W = nullptr;
    cd* Ad = nullptr;
    // non-symmetric elimination: the lower blocks W_jk held as Wt_kj = W_jk^T
    // at the W offsets, and the left coefficients alpha'_jk^T at the alpha offsets
    bool nonsym = false;
    cd* WL = nullptr;
    cd* Bd = nullptr;
    // setup-side low-rank arithmetic (HS_PC_SCHUR_LOWRANK): per pattern entry,
    // the rank of a replaced fill-in block (-1: dense), its V factor, its
    // coefficient block's position in Ad and its ACA rank; the factors live
    // in lrown until the alpha store is built; W holds tcap more elements for
    // the steps' product cores
    bool lowrank = false;
    std::vector<int32_t> lr_rank, lr_rank_aca;
    std::vector<const cd*> lr_v;
    std::vector<int64_t> lr_apos;
    Owned lrown;
    int64_t tcap = 0, xcap = 0;
    int* d_err = nullptr;
    bool d_kept = false;   // D_k written by the elimination (else copied from W in finish)
    // elimination panels: the pattern in CSR (int32), per row the panel column
    // starts (ne + 1 values at rowptr[k] + k), the pair-table offsets, and the
    // Schur output tiles (ti, tj) of every step at tile_ptr[k] .. tile_ptr[k+1]
    std::vector<int32_t> rp32, cols32, pcol;
    std::vector<int64_t> pair_ptr, tile_ptr;
    std::vector<int32_t> panel_m;
    std::vector<std::pair<int16_t, int16_t>> tiles;

    // ordering, symbolic fill, layouts, initial blocks, per-step task lists
    void prepare() {
        P = std::make_unique<hs_precond>();
        P->own.mem = ctx->mem;
        P->H = H;
        P->plan.tree = H->plan.tree;
        P->plan.part = H->plan.part;
        if (opts->kind == HS_PC_BLOCK_JACOBI) {
            // the comparator: no coupling between leaves, natural order, so
            // the setup inverts the diagonal near blocks Z_kk and nothing else
            hs::Partition self;
            for (int64_t l = 0; l < H->nb; ++l) {
                self.near.push_back(l);
                self.near.push_back(l);
            }
            std::vector<int64_t> id(H->nb);
            for (int64_t l = 0; l < H->nb; ++l) id[l] = l;
            P->plan.sym = hs::symbolic(H->nb, self, id);
            P->block_jacobi = true;
        } else {
            P->plan.sym = make_symbolic(H->plan, opts->ordering);
        }
        P->plan.has_sym = true;
        const hs::Symbolic& sy = P->plan.sym;
        const hs::Partition& p = H->plan.part;
        nb = H->nb;
        nnz = sy.nnz();
        P->nb = nb;
        P->bsize.resize(nb);
        P->bstart.resize(nb);
        for (int64_t kk = 0; kk < nb; ++kk) {
            const int64_t ol = sy.order[kk];
            P->bstart[kk] = H->leaf_off[ol];
            P->bsize[kk] = (int32_t)(H->leaf_off[ol + 1] - H->leaf_off[ol]);
        }
        row_of.assign(nnz, 0);
        for (int64_t kk = 0; kk < nb; ++kk)
            for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) row_of[e] = kk;
        // layouts: W diagonal blocks, W pattern blocks, dense alpha, D^-1
        wd_off.assign(nb, 0);
        w_off.assign(nnz, 0);
        ad_off.assign(nnz, 0);
        P->d_off.resize(nb);
        wtot = 0;
        atot = 0;
        dtot = 0;
        for (int64_t kk = 0; kk < nb; ++kk) {
            const int64_t bk = P->bsize[kk];
            wd_off[kk] = wtot;
            wtot += bk * bk;
            P->d_off[kk] = dtot;
            dtot += bk * bk;
            for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) {
                const int64_t bj = P->bsize[sy.cols[e]];
                w_off[e] = wtot;
                wtot += bk * bj;
                ad_off[e] = atot;
                atot += bk * bj;
            }
        }
        P->d_elems = dtot;
        tmp.mem = ctx->mem;
        lowrank = opts->kind == HS_PC_SCHUR_LOWRANK;
        if (lowrank) {
            // bounds over the steps of the product cores (pairs a <= b of
            // S_k at the dense widths) and of the panel (b_k x m_k)
            for (int64_t kk = 0; kk < nb; ++kk) {
                double sj = 0, sj2 = 0;
                for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) {
                    const double bj = P->bsize[sy.cols[e]];
                    sj += bj;
                    sj2 += bj * bj;
                }
                tcap = std::max<int64_t>(tcap, (int64_t)(0.5 * (sj * sj + sj2)));
                xcap = std::max<int64_t>(xcap, (int64_t)(P->bsize[kk] * sj));
            }
            lrown.mem = ctx->mem;
        }
        W = tmp.get<cd>(wtot + tcap);
        Ad = tmp.get<cd>(atot);
        Owned& o = P->own;
        P->d_dinv = o.get<cd>(dtot);
        P->d_D = o.get<cd>(dtot);
        nonsym = opts->kind == HS_PC_SCHUR_NONSYM;
        if (nonsym) {
            WL = tmp.get<cd>(wtot);
            Bd = o.get<cd>(atot);
            P->d_alpha_left = Bd;
            P->alpha_left_elems = atot;
        }
        d_err = tmp.get<int>(1);
        hip_check(hipMemsetAsync(d_err, 0, sizeof(int), s), "memset");
        // scatter Z_N into W (row k of the working matrix = leaf order[k])
        std::map<std::pair<int64_t, int64_t>, int64_t> near_idx;
        for (int64_t e = 0; e < p.n_near(); ++e) near_idx[{p.near[2 * e], p.near[2 * e + 1]}] = e;
        std::vector<hs::CopyTask> init;
        std::vector<hs::CopyTask> init_low;   // Wt_kj = W_jk^T = Z_kj (Z_N is symmetric)
        for (int64_t kk = 0; kk < nb; ++kk) {
            const int64_t ok = sy.order[kk];
            const int32_t bk = P->bsize[kk];
            init.push_back(hs::CopyTask{wd_off[kk], H->near_tasks[near_idx.at({ok, ok})].off, bk, bk, 0, 0});
            for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) {
                const int64_t j = sy.cols[e], oj = sy.order[j];
                const int32_t bj = P->bsize[j];
                if (!sy.orig[e]) {
                    init.push_back(hs::CopyTask{w_off[e], -1, bk, bj, 0, 0});
                } else if (ok < oj) {
                    init.push_back(hs::CopyTask{w_off[e], H->near_tasks[near_idx.at({ok, oj})].off, bk, bj, 0, 0});
                } else {
                    init.push_back(hs::CopyTask{w_off[e], H->near_tasks[near_idx.at({oj, ok})].off, bk, bj, 1, 0});
                }
                if (nonsym) init_low.push_back(init.back());
            }
        }
        hs::CopyTask* d_init = tmp.upload(init, s);
        hs::launch_copy_blocks(d_init, (int64_t)init.size(), H->d_near, W, s);
        hip_check(hipGetLastError(), "k_copy_blocks launch");
        if (nonsym) {
            hs::CopyTask* d_low = tmp.upload(init_low, s);
            hs::launch_copy_blocks(d_low, (int64_t)init_low.size(), H->d_near, WL, s);
            hip_check(hipGetLastError(), "k_copy_blocks launch");
        }
        // elimination panels of every step
        rp32.assign(nb + 1, 0);
        cols32.assign(nnz, 0);
        pcol.assign(nnz + nb, 0);
        pair_ptr.assign(nb + 1, 0);
        tile_ptr.assign(nb + 1, 0);
        panel_m.assign(nb, 0);
        tiles.clear();
        for (int64_t kk = 0; kk < nb; ++kk) {
            const int64_t r0 = sy.rowptr[kk], r1 = sy.rowptr[kk + 1], ne = r1 - r0;
            if (ne > hs::kMaxPattern) fail(HS_EINVAL, "a row of the filled pattern has more than 1024 blocks");
            rp32[kk + 1] = (int32_t)r1;
            int32_t* pc = pcol.data() + r0 + kk;
            pc[0] = 0;
            for (int64_t e = r0; e < r1; ++e) {
                cols32[e] = (int32_t)sy.cols[e];
                pc[e - r0 + 1] = pc[e - r0] + P->bsize[sy.cols[e]];
            }
            const int32_t m = pc[ne];
            panel_m[kk] = m;
            pair_ptr[kk + 1] = pair_ptr[kk] + ne * (ne + 1) / 2;
            schur_tile_list(pc, m, tiles);
            tile_ptr[kk + 1] = (int64_t)tiles.size();
        }
    }

    // The elimination with the setup-side low-rank arithmetic (Sec. 3.4 and
    // the cost argument of Sec. 4), one step at a time. At step k the fill-in
    // blocks W_kj of row k are final; each is compressed by ACA +
    // re-compression at fill_tol (the ranks come back to the host) and, where
    // r (b_k + b_j) < b_k b_j, replaced by U V for everything that follows.
    // The step then works on the compressed panel, [W_kj | U_kj] block by
    // block (width b_j or r):
    //   alpha' = -W_kk^-1 panel (the factor kernel): alpha_kj, or U'_kj with
    //     alpha_kj = U'_kj V_kj;
    //   C' = panel^T alpha' over the pairs a <= b (the Schur tile kernel): a
    //     pair of two dense blocks goes straight into W_ij; any other into a
    //     core T_ab of the compressed shape, which k_core_expand adds to W_ij as
    //     L^T T R (L = V_a or the identity, R = V_b or the identity).
    // A replaced block enters only through these products, so the result is
    // the exact elimination of Z_N + Delta (Delta_kj = U V - W_kj), as in the
    // oracle's definition; FP64 only.
    void eliminate_lowrank() {
        const hs::Symbolic& sy = P->plan.sym;
        lr_rank.assign(nnz, -1);
        lr_rank_aca.assign(nnz, 0);
        lr_v.assign(nnz, nullptr);
        lr_apos.assign(nnz, 0);
        cd* Xp = tmp.get<cd>(std::max<int64_t>(xcap, 1));
        // W offset of pattern entry (i, j), j in S_i (the rows' columns are sorted)
        auto entry = [&](int64_t i, int64_t j) -> int64_t {
            const auto b0 = sy.cols.begin() + sy.rowptr[i], b1 = sy.cols.begin() + sy.rowptr[i + 1];
            const auto it = std::lower_bound(b0, b1, j);
            if (it == b1 || *it != j) fail(HS_EINVAL, "filled pattern is not closed under elimination");
            return (int64_t)(it - sy.cols.begin());
        };
        timed(ctx, HS_KT_ELIM, s, [&] {
            for (int64_t k = 0; k < nb; ++k) {
                Owned st;
                st.mem = ctx->mem;
                const int64_t r0 = sy.rowptr[k];
                const int32_t ne = (int32_t)(sy.rowptr[k + 1] - r0);
                const int32_t bk = P->bsize[k];
                // 1. the final fill-in blocks of row k, compressed
                std::vector<hs::AcaTask> at;
                std::vector<int64_t> fe;
                if (opts->fill_tol > 0.0)
                    for (int32_t a = 0; a < ne; ++a) {
                        const int64_t e = r0 + a;
                        if (sy.orig[e]) continue;
                        hs::AcaTask t{};
                        t.src_off = w_off[e];
                        t.m = bk;
                        t.n = P->bsize[sy.cols[e]];
                        at.push_back(t);
                        fe.push_back(e);
                    }
                LowRankSet set;
                if (!at.empty()) {
                    compress_blocks(lrown, s, at, true, nullptr, 0.0, W, opts->fill_tol, hs::kMaxLeaf, d_err, nullptr,
                                    set, nullptr);
                    check_device_flag(d_err, s);
                }
                std::vector<int32_t> w(ne), rk(ne, -1), bw(ne);
                std::vector<const cd*> up(ne, nullptr), vp(ne, nullptr);
                for (int32_t a = 0; a < ne; ++a) w[a] = bw[a] = P->bsize[sy.cols[r0 + a]];
                for (size_t q = 0; q < fe.size(); ++q) {
                    const int64_t e = fe[q];
                    const int32_t a = (int32_t)(e - r0), r = set.rank[q];
                    lr_rank_aca[e] = set.rank_aca[q];
                    if ((int64_t)r * (bk + bw[a]) < (int64_t)bk * bw[a]) {
                        rk[a] = r;
                        w[a] = r;
                        up[a] = set.ptr[q];
                        vp[a] = set.ptr[q] ? set.ptr[q] + (int64_t)bk * r : nullptr;
                        lr_rank[e] = r;
                        lr_v[e] = vp[a];
                    }
                }
                // 2. the compressed panel: block a at columns [pc[a], pc[a + 1])
                std::vector<int32_t> pc(ne + 1, 0);
                for (int32_t a = 0; a < ne; ++a) pc[a + 1] = pc[a] + w[a];
                const int32_t m = pc[ne];
                if ((int64_t)bk * m > xcap) fail(HS_EINVAL, "compressed panel larger than its bound");
                for (int32_t a = 0; a < ne; ++a) lr_apos[r0 + a] = ad_off[r0] + (int64_t)bk * pc[a];
                std::vector<hs::CopyTask> xc;
                std::vector<hs::ColMajorCopy> uc;
                for (int32_t a = 0; a < ne; ++a) {
                    if (rk[a] < 0) xc.push_back(hs::CopyTask{(int64_t)bk * pc[a], w_off[r0 + a], bk, w[a], 0, 0});
                    else if (rk[a] > 0) uc.push_back(hs::ColMajorCopy{up[a], (int64_t)bk * pc[a], bk, rk[a]});
                }
                // 3. pair table: W targets for dense pairs, cores at wtot + toff for the others
                std::vector<int64_t> pair((size_t)ne * (ne + 1) / 2 + 1, 0);
                std::vector<hs::CopyTask> zc;
                std::vector<hs::CoreExpandTask> ex;
                int64_t toff = 0;
                for (int32_t a = 0; a < ne; ++a) {
                    const int64_t i = sy.cols[r0 + a];
                    for (int32_t b = a; b < ne; ++b) {
                        const int64_t j = sy.cols[r0 + b];
                        const int64_t target = a == b ? wd_off[i] : w_off[entry(i, j)];
                        const int64_t idx = (int64_t)a * ne - (int64_t)a * (a - 1) / 2 - a + b;
                        if (rk[a] < 0 && rk[b] < 0) {
                            pair[idx] = target;
                            continue;
                        }
                        pair[idx] = wtot + toff;
                        const int64_t len = (int64_t)w[a] * w[b];
                        if (len > 0) {
                            zc.push_back(hs::CopyTask{wtot + toff, -1, w[a], w[b], 0, 0});
                            ex.push_back(hs::CoreExpandTask{rk[a] > 0 ? vp[a] : nullptr, rk[b] > 0 ? vp[b] : nullptr, target,
                                                        wtot + toff, bw[a], bw[b], rk[a] > 0 ? rk[a] : 0,
                                                        rk[b] > 0 ? rk[b] : 0});
                        }
                        toff += len;
                    }
                }
                if (toff > tcap) fail(HS_EINVAL, "product cores larger than their bound");
                // the step's flops in factored form (complex multiply-add = 8):
                // inversion, coefficients over the compressed panel, fill-in
                // compression 8 (2 r^2 (b_k + b_j) + r^3) at the ACA rank, core
                // products over pairs a <= b and their expansions
                {
                    double fl = 8.0 / 3.0 * bk * (double)bk * bk + 8.0 * bk * (double)bk * m;
                    for (size_t q = 0; q < fe.size(); ++q) {
                        const double rc = set.rank_aca[q];
                        fl += 8.0 * (2.0 * rc * rc * (bk + at[q].n) + rc * rc * rc);
                    }
                    for (int32_t a = 0; a < ne; ++a)
                        for (int32_t b = a; b < ne; ++b) {
                            fl += 8.0 * w[a] * (double)bk * w[b];
                            const bool la = rk[a] >= 0, lb = rk[b] >= 0;
                            if (la && lb)
                                fl += 8.0 * std::min((double)bw[a] * rk[a] * rk[b] + (double)bw[a] * rk[b] * bw[b],
                                                     (double)rk[a] * rk[b] * bw[b] + (double)bw[a] * rk[a] * bw[b]);
                            else if (la)
                                fl += 8.0 * bw[a] * (double)rk[a] * bw[b];
                            else if (lb)
                                fl += 8.0 * bw[a] * (double)rk[b] * bw[b];
                        }
                    P->flops_factored += fl;
                }
                // 4. tiles: factor tiles over the compressed panel, Schur tiles
                // (ti, tj) holding an element with block(row) <= block(column)
                const int32_t nt = (m + 63) / 64;
                std::vector<hs::ElimTile> ft, stl;
                for (int32_t t = 0; t < std::max<int32_t>(1, nt); ++t) ft.push_back(hs::ElimTile{0, (int16_t)t, -1});
                {
                    std::vector<std::pair<int16_t, int16_t>> tl;
                    schur_tile_list(pc.data(), m, tl);
                    for (const auto& t : tl) stl.push_back(hs::ElimTile{0, t.first, t.second});
                }
                hs::ElimStep es{};
                es.wkk = W + wd_off[k];
                es.dinv = P->d_dinv + P->d_off[k];
                es.x = ne > 0 ? Xp : W;
                es.xs = es.x;
                es.y = ne > 0 ? Ad + ad_off[r0] : Ad;
                es.w = W;
                es.pair = st.upload(pair, s);
                es.pcol = st.upload(pc, s);
                es.err = d_err;
                es.bk = bk;
                es.ne = ne;
                es.m = m;
                es.flags = 0;
                std::vector<hs::ElimStep> esv{es};
                const hs::ElimStep* d_es = st.upload(esv, s);
                hs::launch_copy_blocks(st.upload(xc, s), (int64_t)xc.size(), W, Xp, s);
                hs::launch_copy_colmajor(st.upload(uc, s), (int64_t)uc.size(), Xp, s);
                hs::launch_copy_blocks(st.upload(zc, s), (int64_t)zc.size(), W, W, s);
                timed(ctx, HS_KT_FACTOR, s, [&] {
                    hs::launch_elim_items(d_es, st.upload(ft, s), (int64_t)ft.size(), false, s);
                });
                timed(ctx, HS_KT_SCHUR, s, [&] {
                    hs::launch_elim_items(d_es, st.upload(stl, s), (int64_t)stl.size(), false, s);
                });
                hs::launch_core_expand(st.upload(ex, s), (int64_t)ex.size(), W, s);
                hip_check(hipGetLastError(), "low-rank elimination launches");
                hip_check(hipStreamSynchronize(s), "stream sync");   // the step's tables are freed next
            }
        });
    }

    // after the elimination: D, fill-in compression, the alpha store and the sweep plan
    void finish() {
        const hs::Symbolic& sy = P->plan.sym;
        const hs::Partition& p = H->plan.part;
        Owned& o = P->own;
        (void)p;
        (void)o;
        hip_check(hipGetLastError(), "elimination launches");
        check_device_flag(d_err, s);
        // keep D_k = final W_kk (the persistent elimination has written it)
        if (!d_kept) {
            std::vector<hs::CopyTask> dcp;
            for (int64_t kk = 0; kk < nb; ++kk)
                dcp.push_back(hs::CopyTask{P->d_off[kk], wd_off[kk], P->bsize[kk], P->bsize[kk], 0, 0});
            hs::CopyTask* d_dcp = tmp.upload(dcp, s);
            hs::launch_copy_blocks(d_dcp, (int64_t)dcp.size(), W, P->d_D, s);
        }
        // The sweep plan's layout (chunks, folded ranges, the class of each
        // pattern entry) depends on the symbolic pattern only: a host thread
        // builds it while the fill-in blocks are compressed on the GPU.
        // block -> column of a chunk's range: pairs sorted by block once built
        struct FoldMap {
            std::vector<std::pair<int32_t, int32_t>> kv;
            void set(int32_t k, int32_t v) { kv.emplace_back(k, v); }
            void seal() { std::sort(kv.begin(), kv.end()); }
            int32_t find(int32_t k) const {
                const auto it = std::lower_bound(kv.begin(), kv.end(), std::make_pair(k, INT32_MIN));
                return it != kv.end() && it->first == k ? it->second : -1;
            }
        };
        std::vector<int32_t> chunk_of, loc, wdt, wtt, clast, chunk_first, csize, fwidth, bwidth, fl_n, bl_n;
        std::vector<int64_t> pos, lf_off, lb_off, mf_off, mb_off, cf_off, cb_off, intptr;
        int64_t nch = 0, lft = 0, lbt = 0, mft = 0, mbt = 0, cft = 0, cbt = 0;
        std::vector<FoldMap> ffold, bfold;
        std::vector<int32_t> femap, bemap, fe_off, be_off;
        std::vector<hs::SweepEnt> intent;
        std::vector<hs::ExpandTask> expand;
        std::vector<hs::CopyTask> cfc, cbc;
        std::vector<int64_t> far_f, far_b;   // pushed entries, row-major order
        std::vector<uint8_t> eclass;         // 1: in-chunk or folded entry (a compressed one is expanded)
        std::exception_ptr plan_err;
        std::thread plan_thread([&] {
            try {
                // ---- chunked sweep plan: consecutive block rows grouped up to kMaxChunk points
                chunk_of.assign(nb, 0);
                loc.assign(nb, 0);
                wdt.assign(nb, 0);
                wtt.assign(nb, 0);
                clast.assign(nb, 0);
                pos.assign(nb, 0);
                {
                    int64_t pp = 0;
                    int32_t cur = -1, used = chunk_lim;
                    for (int64_t kk = 0; kk < nb; ++kk) {
                        const int32_t bk = P->bsize[kk];
                        if (used + bk > chunk_lim) {
                            ++cur;
                            used = 0;
                            chunk_first.push_back((int32_t)kk);
                        }
                        chunk_of[kk] = cur;
                        loc[kk] = used;
                        used += bk;
                        wdt[kk] = used;
                        pos[kk] = pp;
                        pp += bk;
                    }
                    chunk_first.push_back((int32_t)nb);
                }
                nch = (int64_t)chunk_first.size() - 1;
                P->nchunk = nch;
                csize.assign(nch, 0);
                for (int64_t c = 0; c < nch; ++c) {
                    int32_t sz = 0;
                    for (int32_t kk = chunk_first[c]; kk < chunk_first[c + 1]; ++kk) sz += P->bsize[kk];
                    csize[c] = sz;
                    for (int32_t kk = chunk_first[c]; kk < chunk_first[c + 1]; ++kk) {
                        clast[kk] = chunk_first[c + 1] - 1;
                        wtt[kk] = sz - loc[kk];
                    }
                }
                // Folded neighbour ranges. Forward, chunk c: all of chunk c-1 (contiguous),
                // then the source blocks of chunks <= c-2 coupled to chunk c, nearest chunk
                // first, while they fit in fold_cols columns; the entries of the source
                // blocks left out are pushed. Backward mirrored (chunk c+1, then >= c+2).
                fwidth.assign(nch, 0);
                bwidth.assign(nch, 0);
                fl_n.assign(nch, 0);
                bl_n.assign(nch, 0);
                ffold.assign(nch, FoldMap{});
                bfold.assign(nch, FoldMap{});
                fe_off.assign(nch + 1, 0);
                be_off.assign(nch + 1, 0);
                {
                    std::vector<std::vector<int32_t>> fsrc(nch), bsrc(nch);
                    for (int64_t kk = 0; kk < nb; ++kk)
                        for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) {
                            const int32_t j = (int32_t)sy.cols[e];
                            const int32_t ck = chunk_of[kk], cj = chunk_of[j];
                            if (cj >= ck + 2) {
                                fsrc[cj].push_back((int32_t)kk);
                                bsrc[ck].push_back(j);
                            }
                        }
                    auto uniq = [](std::vector<int32_t>& v) {
                        std::sort(v.begin(), v.end());
                        v.erase(std::unique(v.begin(), v.end()), v.end());
                    };
                    for (int64_t c = 0; c < nch; ++c) {
                        uniq(fsrc[c]);
                        uniq(bsrc[c]);
                        // nearest chunk first, blocks ascending within a chunk
                        std::stable_sort(fsrc[c].begin(), fsrc[c].end(),
                                         [&](int32_t x, int32_t y) { return chunk_of[x] > chunk_of[y]; });
                        std::stable_sort(bsrc[c].begin(), bsrc[c].end(),
                                         [&](int32_t x, int32_t y) { return chunk_of[x] < chunk_of[y]; });
                        fe_off[c] = (int32_t)femap.size();
                        if (c > 0) {
                            int32_t cols = 0;
                            for (int32_t kk = chunk_first[c - 1]; kk < chunk_first[c]; ++kk) {
                                ffold[c].set(kk, cols);
                                cols += P->bsize[kk];
                            }
                            fl_n[c] = cols;
                            for (int32_t kk : fsrc[c]) {
                                if (cols + P->bsize[kk] > fold_cols) break;
                                ffold[c].set(kk, cols);
                                for (int32_t q = 0; q < P->bsize[kk]; ++q) femap.push_back((int32_t)(pos[kk] + q));
                                cols += P->bsize[kk];
                            }
                            fwidth[c] = cols;
                        }
                        be_off[c] = (int32_t)bemap.size();
                        if (c + 1 < nch) {
                            int32_t cols = 0;
                            for (int32_t kk = chunk_first[c + 1]; kk < chunk_first[c + 2]; ++kk) {
                                bfold[c].set(kk, cols);
                                cols += P->bsize[kk];
                            }
                            bl_n[c] = cols;
                            for (int32_t kk : bsrc[c]) {
                                if (cols + P->bsize[kk] > fold_cols) break;
                                bfold[c].set(kk, cols);
                                for (int32_t q = 0; q < P->bsize[kk]; ++q) bemap.push_back((int32_t)(pos[kk] + q));
                                cols += P->bsize[kk];
                            }
                            bwidth[c] = cols;
                        }
                    }
                    fe_off[nch] = (int32_t)femap.size();
                    be_off[nch] = (int32_t)bemap.size();
                    for (int64_t c = 0; c < nch; ++c) {
                        ffold[c].seal();
                        bfold[c].seal();
                    }
                }
                lf_off.assign(nb, 0);
                lb_off.assign(nb, 0);
                mf_off.assign(nb, 0);
                mb_off.assign(nb, 0);
                cf_off.assign(nch, -1);
                cb_off.assign(nch, -1);
                for (int64_t kk = 0; kk < nb; ++kk) {
                    const int64_t bk = P->bsize[kk], c = chunk_of[kk];
                    lf_off[kk] = lft;
                    lft += bk * wdt[kk];
                    lb_off[kk] = lbt;
                    lbt += bk * wtt[kk];
                    mf_off[kk] = mft;
                    mft += bk * fwidth[c];
                    mb_off[kk] = mbt;
                    mbt += bk * bwidth[c];
                }
                for (int64_t c = 0; c < nch; ++c) {
                    cf_off[c] = cft;
                    cft += (int64_t)csize[c] * fwidth[c];
                    cb_off[c] = cbt;
                    cbt += (int64_t)csize[c] * bwidth[c];
                }
                P->linv_elems = lft + lbt + mft + mbt;
                // entries: in-chunk ones feed Linv, folded ones the coupling products of
                // their target chunk, the rest are pushed from their source block into
                // per-entry slots (separately per direction)
                intptr.assign(nb + 1, 0);
                for (int64_t e = 0; e < nnz; ++e)
                    if (chunk_of[row_of[e]] == chunk_of[sy.cols[e]]) intptr[sy.cols[e] + 1]++;
                for (int64_t j = 0; j < nb; ++j) intptr[j + 1] += intptr[j];
                intent.assign(intptr[nb], hs::SweepEnt{});
                eclass.assign(nnz, 0);
                {
                    std::vector<int64_t> fi(intptr.begin(), intptr.end() - 1);
                    for (int64_t kk = 0; kk < nb; ++kk)
                        for (int64_t e = sy.rowptr[kk]; e < sy.rowptr[kk + 1]; ++e) {
                            const int32_t j = (int32_t)sy.cols[e];
                            const int32_t ck = chunk_of[kk], cj = chunk_of[j];
                            const int32_t bk = P->bsize[kk], bj = P->bsize[j];
                            const bool in_chunk = cj == ck;
                            const int32_t fcol = in_chunk ? -1 : ffold[cj].find((int32_t)kk);
                            const int32_t bcol = in_chunk ? -1 : bfold[ck].find(j);
                            const bool ffolded = fcol >= 0;
                            const bool bfolded = bcol >= 0;
                            if (in_chunk || ffolded || bfolded) eclass[e] = 1;
                            if (in_chunk) {
                                intent[fi[j]++] = hs::SweepEnt{ad_off[e], (int32_t)kk, -1};
                                continue;
                            }
                            // forward coupling of chunk cj: rows of block j, columns of block k (alpha_kj^T)
                            if (ffolded)
                                cfc.push_back(hs::CopyTask{cf_off[cj] + (int64_t)loc[j] * fwidth[cj] + fcol, ad_off[e],
                                                           bj, bk, 1, fwidth[cj]});
                            else
                                far_f.push_back(e);
                            // backward coupling of chunk ck: rows of block k, columns of block j (alpha_kj)
                            if (bfolded)
                                cbc.push_back(hs::CopyTask{cb_off[ck] + (int64_t)loc[kk] * bwidth[ck] + bcol, ad_off[e],
                                                           bk, bj, 0, bwidth[ck]});
                            else
                                far_b.push_back(e);
                        }
                }
            } catch (...) {
                plan_err = std::current_exception();
            }
        });
        struct PlanJoiner {
            std::thread& th;
            ~PlanJoiner() {
                if (th.joinable()) th.join();
            }
        } plan_join{plan_thread};
        // fill-in compression (Sec. 3.4)
        std::vector<int64_t> fill_e;
        for (int64_t e = 0; e < nnz; ++e)
            if (!sy.orig[e]) fill_e.push_back(e);
        P->n_fill = (int64_t)fill_e.size();
        P->a_rank.assign(nnz, -1);
        LowRankSet fills;
        std::vector<char> keep(fill_e.size(), 0);
        if (lowrank) {
            // the coefficient blocks as the low-rank elimination left them: a
            // dense block in its row's compressed panel, or U' there (b_k x r,
            // row-major) with V from the fill-in compression
            P->a_off.resize(nnz);
            int64_t ftot = 0;
            for (int64_t e = 0; e < nnz; ++e) {
                P->a_rank[e] = lr_rank[e];
                P->a_off[e] = ftot;
                const int64_t bk = P->bsize[row_of[e]], bj = P->bsize[sy.cols[e]];
                ftot += lr_rank[e] >= 0 ? (int64_t)lr_rank[e] * (bk + bj) : bk * bj;
                if (lr_rank[e] >= 0) ++P->n_lowrank;
                const double rr = lr_rank_aca[e];
                P->flops_fill += rr * rr * (double)(bk + bj);
            }
            P->alpha_elems = ftot;
            P->d_alpha = o.get<cd>(std::max<int64_t>(ftot, 1));
            std::vector<hs::CopyTask> cp;
            std::vector<hs::PtrCopy> vc;
            for (int64_t e = 0; e < nnz; ++e) {
                const int32_t bk = P->bsize[row_of[e]], bj = P->bsize[sy.cols[e]], r = lr_rank[e];
                if (r < 0) {
                    cp.push_back(hs::CopyTask{P->a_off[e], lr_apos[e], bk, bj, 0, 0});
                } else if (r > 0) {
                    // column-major b_k x r = row-major r x b_k, from the row-major b_k x r panel block
                    cp.push_back(hs::CopyTask{P->a_off[e], lr_apos[e], r, bk, 1, 0});
                    vc.push_back(hs::PtrCopy{lr_v[e], P->a_off[e] + (int64_t)bk * r, (int64_t)r * bj});
                }
            }
            hs::CopyTask* d_cp = tmp.upload(cp, s);
            hs::launch_copy_blocks(d_cp, (int64_t)cp.size(), Ad, P->d_alpha, s);
            hs::PtrCopy* d_vc = tmp.upload(vc, s);
            hs::launch_copy_ptrs(d_vc, (int64_t)vc.size(), P->d_alpha, s);
            // the sweep plan below reads the dense coefficient blocks at their
            // dense positions in Ad (the low-rank ones it expands from the
            // store): put them back there from the store
            std::vector<hs::CopyTask> back;
            for (int64_t e = 0; e < nnz; ++e)
                if (lr_rank[e] < 0)
                    back.push_back(hs::CopyTask{ad_off[e], P->a_off[e], P->bsize[row_of[e]], P->bsize[sy.cols[e]], 0, 0});
            hs::CopyTask* d_back = tmp.upload(back, s);
            hs::launch_copy_blocks(d_back, (int64_t)back.size(), P->d_alpha, Ad, s);
            hip_check(hipStreamSynchronize(s), "stream sync");
            lrown.release();
        } else if (opts->fill_tol > 0.0 && !fill_e.empty()) {
            std::vector<hs::AcaTask> ft;
            for (int64_t e : fill_e) {
                hs::AcaTask a{};
                a.src_off = ad_off[e];
                a.m = P->bsize[row_of[e]];
                a.n = P->bsize[sy.cols[e]];
                ft.push_back(a);
            }
            // compress into a temporary owner; kept blocks are copied to the final store
            Owned lr;
            lr.mem = ctx->mem;
            compress_blocks(lr, s, ft, true, nullptr, 0.0, Ad, opts->fill_tol, hs::kMaxLeaf, d_err, nullptr, fills,
                            nullptr);
            check_device_flag(d_err, s);
            for (size_t q = 0; q < fill_e.size(); ++q) {
                const int64_t bk = ft[q].m, bj = ft[q].n, r = fills.rank[q];
                keep[q] = (r * (bk + bj) < bk * bj) ? 1 : 0;
                if (keep[q]) P->a_rank[fill_e[q]] = (int)r;
                const double rr = fills.rank_aca[q];
                P->flops_fill += rr * rr * (double)(bk + bj);
            }
            // final alpha store
            P->a_off.resize(nnz);
            int64_t ftot = 0;
            for (int64_t e = 0; e < nnz; ++e) {
                P->a_off[e] = ftot;
                const int64_t bk = P->bsize[row_of[e]], bj = P->bsize[sy.cols[e]];
                ftot += P->a_rank[e] >= 0 ? (int64_t)P->a_rank[e] * (bk + bj) : bk * bj;
            }
            P->alpha_elems = ftot;
            P->d_alpha = o.get<cd>(std::max<int64_t>(ftot, 1));
            std::vector<hs::CopyTask> cp;
            for (int64_t e = 0; e < nnz; ++e)
                if (P->a_rank[e] < 0)
                    cp.push_back(hs::CopyTask{P->a_off[e], ad_off[e], P->bsize[row_of[e]], P->bsize[sy.cols[e]], 0, 0});
            hs::CopyTask* d_cp = tmp.upload(cp, s);
            hs::launch_copy_blocks(d_cp, (int64_t)cp.size(), Ad, P->d_alpha, s);
            std::vector<hs::PtrCopy> pc;
            for (size_t q = 0; q < fill_e.size(); ++q) {
                const int64_t e = fill_e[q];
                if (!keep[q]) continue;
                const int64_t cnt = (int64_t)P->a_rank[e] * (ft[q].m + ft[q].n);
                if (cnt) pc.push_back(hs::PtrCopy{fills.ptr[q], P->a_off[e], cnt});
                ++P->n_lowrank;
            }
            hs::PtrCopy* d_pc = tmp.upload(pc, s);
            hs::launch_copy_ptrs(d_pc, (int64_t)pc.size(), P->d_alpha, s);
            hip_check(hipStreamSynchronize(s), "stream sync");
        } else {
            P->a_off = ad_off;
            P->alpha_elems = atot;
            P->d_alpha = o.get<cd>(std::max<int64_t>(atot, 1));
            hip_check(hipMemcpyAsync(P->d_alpha, Ad, atot * 16, hipMemcpyDeviceToDevice, s), "D2D");
        }
        plan_thread.join();
        if (plan_err) std::rethrow_exception(plan_err);
        for (int64_t e = 0; e < nnz; ++e)
            if (eclass[e] && P->a_rank[e] >= 0)
                expand.push_back(hs::ExpandTask{P->a_off[e], ad_off[e], P->bsize[row_of[e]], P->bsize[sy.cols[e]],
                                                P->a_rank[e], 0});
        // push lists (grouped by source chunk) and per-target gather lists
        std::vector<hs::PushEnt> fpush, bpush;
        std::vector<int32_t> fgrp, fgrp_n, bgrp, bgrp_n;
        std::vector<int64_t> fgptr(nb + 1, 0), bgptr(nb + 1, 0), fgslot, bgslot;
        std::vector<std::vector<int32_t>> fgrp_of(nch), bgrp_of(nch);   // group ids per source chunk
        {
            // forward: source k (rows ascending = sources ascending); backward: source j
            std::vector<int64_t> fo(far_f), bo(far_b);
            std::stable_sort(fo.begin(), fo.end(), [&](int64_t x, int64_t y) {
                return row_of[x] != row_of[y] ? row_of[x] < row_of[y] : sy.cols[x] < sy.cols[y];
            });
            std::stable_sort(bo.begin(), bo.end(), [&](int64_t x, int64_t y) {
                return sy.cols[x] != sy.cols[y] ? sy.cols[x] < sy.cols[y] : row_of[x] < row_of[y];
            });
            std::vector<int64_t> fslot(nnz, -1), bslot(nnz, -1);
            int64_t fs = 0, bs = 0;
            for (int64_t e : fo) {
                fslot[e] = fs;
                fs += P->bsize[sy.cols[e]];
            }
            for (int64_t e : bo) {
                bslot[e] = bs;
                bs += P->bsize[row_of[e]];
            }
            // push order: by source chunk, then the target chunk needed soonest
            // (forward the lowest, backward the highest), then source and target
            std::vector<int64_t> fpo(far_f), bpo(far_b);
            std::stable_sort(fpo.begin(), fpo.end(), [&](int64_t x, int64_t y) {
                const int32_t sx = chunk_of[row_of[x]], sy_ = chunk_of[row_of[y]];
                if (sx != sy_) return sx < sy_;
                const int32_t tx = chunk_of[sy.cols[x]], ty = chunk_of[sy.cols[y]];
                if (tx != ty) return tx < ty;
                return row_of[x] != row_of[y] ? row_of[x] < row_of[y] : sy.cols[x] < sy.cols[y];
            });
            std::stable_sort(bpo.begin(), bpo.end(), [&](int64_t x, int64_t y) {
                const int32_t sx = chunk_of[sy.cols[x]], sy_ = chunk_of[sy.cols[y]];
                if (sx != sy_) return sx < sy_;
                const int32_t tx = chunk_of[row_of[x]], ty = chunk_of[row_of[y]];
                if (tx != ty) return tx > ty;
                return sy.cols[x] != sy.cols[y] ? sy.cols[x] < sy.cols[y] : row_of[x] < row_of[y];
            });
            for (int64_t e : fpo)
                fpush.push_back(hs::PushEnt{P->a_off[e], fslot[e], (int32_t)row_of[e], (int32_t)sy.cols[e],
                                            P->a_rank[e], 0});
            for (int64_t e : bpo)
                bpush.push_back(hs::PushEnt{P->a_off[e], bslot[e], (int32_t)sy.cols[e], (int32_t)row_of[e],
                                            P->a_rank[e], 0});
            P->fslot_total = fs;
            P->bslot_total = bs;
            auto groups = [&](const std::vector<hs::PushEnt>& lst, std::vector<int32_t>& grp, std::vector<int32_t>& grpn,
                              std::vector<std::vector<int32_t>>& of) {
                size_t q = 0;
                while (q < lst.size()) {
                    const int32_t c = chunk_of[lst[q].src];
                    size_t r = q;
                    while (r < lst.size() && r - q < (size_t)hs::kPushGroup && chunk_of[lst[r].src] == c) ++r;
                    of[c].push_back((int32_t)grp.size());
                    grp.push_back((int32_t)q);
                    grpn.push_back((int32_t)(r - q));
                    q = r;
                }
            };
            groups(fpush, fgrp, fgrp_n, fgrp_of);
            groups(bpush, bgrp, bgrp_n, bgrp_of);
            // gather lists: forward target j sums its slots by ascending source k; backward target k by ascending j
            for (int64_t e : fo) fgptr[sy.cols[e] + 1]++;
            for (int64_t e : bo) bgptr[row_of[e] + 1]++;
            for (int64_t x = 0; x < nb; ++x) {
                fgptr[x + 1] += fgptr[x];
                bgptr[x + 1] += bgptr[x];
            }
            fgslot.resize(fgptr[nb]);
            bgslot.resize(bgptr[nb]);
            std::vector<int64_t> ff(fgptr.begin(), fgptr.end() - 1), bf(bgptr.begin(), bgptr.end() - 1);
            for (int64_t e : fo) fgslot[ff[sy.cols[e]]++] = fslot[e];   // fo is sorted by source k
            std::vector<int64_t> bo2(far_b);   // backward targets gather by ascending source j
            std::stable_sort(bo2.begin(), bo2.end(), [&](int64_t x, int64_t y) {
                return row_of[x] != row_of[y] ? row_of[x] < row_of[y] : sy.cols[x] < sy.cols[y];
            });
            for (int64_t e : bo2) bgslot[bf[row_of[e]]++] = bslot[e];
        }
        P->d_bstart = o.upload(P->bstart, s);
        P->d_bsize = o.upload(P->bsize, s);
        P->d_dinv_off = o.upload(P->d_off, s);
        hs::SweepPlan& sp = P->sp;
        sp.nb = (int)nb;
        sp.nch = (int)nch;
        sp.bmax = *std::max_element(P->bsize.begin(), P->bsize.end());
        sp.chunk_of = o.upload(chunk_of, s);
        sp.csize = o.upload(csize, s);
        sp.n = H->n;
        sp.bstart = P->d_bstart;
        sp.bsize = P->d_bsize;
        sp.pos = o.upload(pos, s);
        sp.loc = o.upload(loc, s);
        sp.w = o.upload(wdt, s);
        sp.wt = o.upload(wtt, s);
        sp.clast = o.upload(clast, s);
        sp.lf_off = o.upload(lf_off, s);
        sp.lb_off = o.upload(lb_off, s);
        sp.mf_off = o.upload(mf_off, s);
        sp.mb_off = o.upload(mb_off, s);
        cd* d_lf = o.get<cd>(std::max<int64_t>(lft, 1));
        cd* d_lb = o.get<cd>(std::max<int64_t>(lbt, 1));
        cd* d_mf = o.get<cd>(std::max<int64_t>(mft, 1));
        cd* d_mb = o.get<cd>(std::max<int64_t>(mbt, 1));
        sp.lf = d_lf;
        sp.lb = d_lb;
        sp.mf = d_mf;
        sp.mb = d_mb;
        sp.fpush = o.upload(fpush, s);
        sp.fgrp = o.upload(fgrp, s);
        sp.fgrp_n = o.upload(fgrp_n, s);
        sp.fgptr = o.upload(fgptr, s);
        sp.fgslot = o.upload(fgslot, s);
        {
            // backward pushes of dense entries read alpha_kj^T (b_j x b_k row-major),
            // so they run as column sums like the forward ones
            std::vector<hs::CopyTask> tc;
            int64_t tt = 0;
            for (auto& e : bpush)
                if (e.rank < 0) {
                    const int32_t bk = P->bsize[e.dst], bj = P->bsize[e.src];
                    tc.push_back(hs::CopyTask{tt, e.aoff, bj, bk, 1, 0});
                    e.aoff = tt;
                    tt += (int64_t)bk * bj;
                }
            cd* d_at = o.get<cd>(std::max<int64_t>(tt, 1));
            P->alpha_t_elems = tt;
            hs::CopyTask* d_tc = tmp.upload(tc, s);
            hs::launch_copy_blocks(d_tc, (int64_t)tc.size(), P->d_alpha, d_at, s);
            sp.alpha_t = d_at;
        }
        sp.bpush = o.upload(bpush, s);
        sp.bgrp = o.upload(bgrp, s);
        sp.bgrp_n = o.upload(bgrp_n, s);
        sp.bgptr = o.upload(bgptr, s);
        sp.bgslot = o.upload(bgslot, s);
        sp.alpha = P->d_alpha;
        sp.dinv = P->d_dinv;
        sp.dinv_off = P->d_dinv_off;
        // compressed blocks inside a chunk or between neighbouring chunks enter the dense
        // products as their U V product (the same operator as the rest of the apply)
        hs::ExpandTask* d_exp = tmp.upload(expand, s);
        hs::launch_lr_expand(d_exp, (int64_t)expand.size(), P->d_alpha, Ad, s);
        int32_t* d_cf = tmp.upload(chunk_first, s);
        int64_t* d_ip = tmp.upload(intptr, s);
        hs::SweepEnt* d_ie = tmp.upload(intent, s);
        hs::launch_linv(sp, (int)nch, d_cf, d_ip, d_ie, Ad, d_lf, s);
        hs::launch_linv_transpose(sp, d_lb, s);
        // coupling matrices and their products with Linv / Linv^T
        cd* d_C = tmp.get<cd>(std::max<int64_t>(cft + cbt, 1));
        hip_check(hipMemsetAsync(d_C, 0, sizeof(cd) * std::max<int64_t>(cft + cbt, 1), s), "memset");
        for (auto& t : cbc) t.dst_off += cft;
        hs::CopyTask* d_cfc = tmp.upload(cfc, s);
        hs::CopyTask* d_cbc = tmp.upload(cbc, s);
        hs::launch_copy_blocks(d_cfc, (int64_t)cfc.size(), Ad, d_C, s);
        hs::launch_copy_blocks(d_cbc, (int64_t)cbc.size(), Ad, d_C, s);
        // M_f = Linv C_f and M_b = Linv^T C_b per chunk, by 64 x 64 output tiles
        // over the chunk's rows: a row of block k covers chunk columns
        // [0, loc_k + b_k) forward and [loc_k, csize) backward
        std::vector<hs::ChunkRow> rf(H->n), rb(H->n);
        std::vector<hs::ChunkTile> tf, tb;
        for (int64_t kk = 0; kk < nb; ++kk) {
            const int32_t c = chunk_of[kk], bk = P->bsize[kk];
            const int64_t r0 = pos[chunk_first[c]] + loc[kk];
            for (int32_t a = 0; a < bk; ++a) {
                rf[r0 + a] = hs::ChunkRow{lf_off[kk] + (int64_t)a * wdt[kk], mf_off[kk] + (int64_t)a * fwidth[c], 0,
                                          wdt[kk]};
                rb[r0 + a] = hs::ChunkRow{lb_off[kk] + (int64_t)a * wtt[kk], mb_off[kk] + (int64_t)a * bwidth[c],
                                          loc[kk], wtt[kk]};
            }
        }
        for (int64_t c = 0; c < nch; ++c) {
            const int32_t base = (int32_t)pos[chunk_first[c]], cs = csize[c];
            for (int32_t t0 = 0; t0 < cs; t0 += 64) {
                const int32_t nr = std::min(64, cs - t0);
                const hs::ChunkRow& last = rf[base + t0 + nr - 1];
                const hs::ChunkRow& first = rb[base + t0];
                for (int32_t c0 = 0; c0 < fwidth[c]; c0 += 64)
                    tf.push_back(hs::ChunkTile{cf_off[c], base + t0, nr, c0, fwidth[c], 0, last.k0 + last.kw});
                for (int32_t c0 = 0; c0 < bwidth[c]; c0 += 64)
                    tb.push_back(hs::ChunkTile{cft + cb_off[c], base + t0, nr, c0, bwidth[c], first.k0, cs});
            }
        }
        hs::ChunkRow* d_rf = tmp.upload(rf, s);
        hs::ChunkRow* d_rb = tmp.upload(rb, s);
        hs::ChunkTile* d_tf = tmp.upload(tf, s);
        hs::ChunkTile* d_tb = tmp.upload(tb, s);
        hs::launch_chunk_gemm(d_tf, (int64_t)tf.size(), d_rf, d_lf, d_C, d_mf, s);
        hs::launch_chunk_gemm(d_tb, (int64_t)tb.size(), d_rb, d_lb, d_C, d_mb, s);
        hip_check(hipGetLastError(), "linv launches");
        // Row workers: per chunk its ranges, per point row its matrix slices.
        // Work items of the other workgroups in dependency order: per chunk its
        // block rows (phase A), then the pushes from the chunk before it;
        // forward ascending, backward descending.
        {
            std::vector<hs::SweepChunk> fch(nch), bch(nch);
            std::vector<hs::RowTask> frow(H->n), brow(H->n);
            for (int64_t c = 0; c < nch; ++c) {
                const int32_t pc = (int32_t)pos[chunk_first[c]], nc = csize[c];
                const int32_t nbk = chunk_first[c + 1] - chunk_first[c];
                hs::SweepChunk f{};
                f.pc = pc;
                f.nc = nc;
                f.nblocks = nbk;
                if (c > 0) {
                    f.w2 = fwidth[c];
                    f.l_n = fl_n[c];
                    f.l_g = (int32_t)pos[chunk_first[c - 1]];
                    f.e_n = f.w2 - f.l_n;
                    f.e_off = fe_off[c];
                    f.need1 = csize[c - 1];
                    f.need2 = c >= 2 ? csize[c - 2] : 0;
                    f.need3 = c >= 3 ? csize[c - 3] : 0;
                }
                fch[c] = f;
                hs::SweepChunk b{};
                b.pc = pc;
                b.nc = nc;
                b.nblocks = nbk;
                if (c + 1 < nch) {
                    b.w2 = bwidth[c];
                    b.l_n = bl_n[c];
                    b.l_g = pc + nc;
                    b.e_n = b.w2 - b.l_n;
                    b.e_off = be_off[c];
                    b.need1 = csize[c + 1];
                    b.need2 = c + 2 < nch ? csize[c + 2] : 0;
                    b.need3 = c + 3 < nch ? csize[c + 3] : 0;
                }
                bch[c] = b;
                for (int32_t kk = chunk_first[c]; kk < chunk_first[c + 1]; ++kk)
                    for (int32_t r = 0; r < P->bsize[kk]; ++r) {
                        const int64_t i = pos[kk] + r;
                        frow[i] = hs::RowTask{lf_off[kk] + (int64_t)r * wdt[kk], mf_off[kk] + (int64_t)r * fwidth[c],
                                              wdt[kk], 0, (int32_t)(P->bstart[kk] + r), 0};
                        brow[i] = hs::RowTask{lb_off[kk] + (int64_t)r * wtt[kk], mb_off[kk] + (int64_t)r * bwidth[c],
                                              wtt[kk], loc[kk], (int32_t)(P->bstart[kk] + r), 0};
                    }
            }
            std::vector<int32_t> fwd, bwd;
            for (int64_t t = 0; t <= nch; ++t) {
                if (t < nch)
                    for (int32_t kk = chunk_first[t]; kk < chunk_first[t + 1]; ++kk) fwd.push_back(kk);
                if (t >= 1)
                    for (int32_t g : fgrp_of[t - 1]) fwd.push_back((int32_t)nb + g);
            }
            for (int64_t t = 0; t <= nch; ++t) {
                const int64_t c = nch - 1 - t;
                if (c >= 0)
                    for (int32_t kk = chunk_first[c + 1] - 1; kk >= chunk_first[c]; --kk) bwd.push_back(kk);
                if (t >= 1)
                    for (int32_t g : bgrp_of[c + 1]) bwd.push_back((int32_t)nb + g);
            }
            P->items.nfwd = (int64_t)fwd.size();
            P->items.nbwd = (int64_t)bwd.size();
            P->items.fwd = o.upload(fwd, s);
            P->items.bwd = o.upload(bwd, s);
            P->items.fchunk = o.upload(fch, s);
            P->items.bchunk = o.upload(bch, s);
            P->items.frow = o.upload(frow, s);
            P->items.brow = o.upload(brow, s);
            P->items.femap = o.upload(femap, s);
            P->items.bemap = o.upload(bemap, s);
        }
        if (opts->precision == HS_PREC_MIXED) {
            // the same plan over complex64 copies of every matrix the apply reads
            static_assert(sizeof(hs::SweepPlanT<hs::cf>) == sizeof(hs::SweepPlan), "plans differ only in types");
            std::memcpy(static_cast<void*>(&P->sp32), &sp, sizeof(sp));
            P->sp32.lf = c64_copy(o, tmp, sp.lf, lft, s);
            P->sp32.lb = c64_copy(o, tmp, sp.lb, lbt, s);
            P->sp32.mf = c64_copy(o, tmp, sp.mf, mft, s);
            P->sp32.mb = c64_copy(o, tmp, sp.mb, mbt, s);
            P->sp32.alpha = c64_copy(o, tmp, sp.alpha, P->alpha_elems, s);
            P->sp32.alpha_t = c64_copy(o, tmp, sp.alpha_t, P->alpha_t_elems, s);
            P->sp32.dinv = c64_copy(o, tmp, sp.dinv, P->d_elems, s);
            P->c64 = true;
        }
        hip_check(hipStreamSynchronize(s), "stream sync");
        tmp.release();
        hs_info info;
        fill_info_plan(P->plan, &info);
        P->flops_setup = info.flops_setup;
        P->max_dk = info.max_dk;
    }
};

// The elimination of every job (Eq. 14, 19: invert W_kk, alpha_kj =
// -W_kk^-1 W_kj, W_ij += W_ki^T alpha_kj).
//
// Components of the leaf graph have separate elimination trees (every block
// of S_k is an ancestor of k), so their steps read and write disjoint blocks,
// while the steps of one component k_1, k_2, ... keep their order. Each entry
// (a step; the non-symmetric elimination has two per non-empty row)
// contributes factor tiles F (one per 64 panel columns, at least one) and
// Schur tiles S. Per component the launches are
//   {F(k_1)}, then for each i: {F(k_i+1), S(k_i)} when step k_i+1 takes the
//   look-ahead (S_{k_i} starts with k_i+1: its factor tiles apply k_i's update
//   of row k_i+1 themselves and k_i's Schur tiles skip that row), else
//   {S(k_i)}, {F(k_i+1)};
// launch g runs the g-th group of every component. Every item's inputs come
// from earlier launches, so one kernel boundary per group orders the steps,
// and with the look-ahead the inversion chain waits for no Schur launch.
// (One persistent launch with device-side readiness counters, tried instead,
// was slower: its blocks handed between workgroups needed device-scope loads
// and stores, which made each Schur tile about twice as slow, 71.7 ms against
// 59.6 ms on c2.)
void eliminate(std::vector<SetupJob*>& jobs, hipStream_t s) {
    Owned tmp;
    tmp.mem = jobs.front()->ctx->mem;
    std::vector<hs::ElimStep> es;
    std::vector<std::vector<int32_t>> sidx;   // per job and step: its (upper) entry in es
    std::vector<std::vector<int32_t>> lamap_h(jobs.size());
    std::vector<int32_t*> lamap_d(jobs.size());
    for (size_t q = 0; q < jobs.size(); ++q) {
        SetupJob* j = jobs[q];
        hs_precond* P = j->P.get();
        const hs::Symbolic& sy = P->plan.sym;
        const int32_t* d_rp = tmp.upload(j->rp32, s);
        const int32_t* d_cols = tmp.upload(j->cols32, s);
        const int64_t* d_woff = tmp.upload(j->w_off, s);
        const int64_t* d_wdoff = tmp.upload(j->wd_off, s);
        const int32_t* d_pcol = tmp.upload(j->pcol, s);
        lamap_h[q].assign(std::max<size_t>(j->cols32.size(), 1), -1);
        lamap_d[q] = tmp.get<int32_t>(lamap_h[q].size());
        int64_t* d_pair = tmp.get<int64_t>(std::max<int64_t>(j->pair_ptr[j->nb], 1));
        std::vector<hs::PairStep> ps;
        sidx.emplace_back(j->nb);
        for (int64_t k = 0; k < j->nb; ++k) {
            const int64_t r0 = sy.rowptr[k];
            const int32_t ne = (int32_t)(sy.rowptr[k + 1] - r0);
            if (ne > 0) ps.push_back(hs::PairStep{d_cols + r0, d_rp, d_cols, d_woff, d_wdoff, d_pair + j->pair_ptr[k], ne, 0});
            hs::ElimStep e{};
            e.wkk = j->W + j->wd_off[k];
            e.dinv = P->d_dinv + P->d_off[k];
            e.x = ne > 0 ? j->W + j->w_off[r0] : j->W;
            e.xs = j->nonsym && ne > 0 ? j->WL + j->w_off[r0] : e.x;
            e.y = ne > 0 ? j->Ad + j->ad_off[r0] : j->Ad;
            e.w = j->W;
            e.pair = d_pair + j->pair_ptr[k];
            e.pcol = d_pcol + r0 + k;
            e.err = j->d_err;
            e.bk = P->bsize[k];
            e.ne = ne;
            e.m = j->panel_m[k];
            e.flags = 0;
            e.dfin = P->d_D + P->d_off[k];
            e.lamap = lamap_d[q] + r0;
            e.prev = -1;
            sidx.back()[k] = (int32_t)es.size();
            es.push_back(e);
            if (j->nonsym && ne > 0) {
                // the left coefficients and the lower triangle's updates
                hs::ElimStep l = e;
                l.x = e.xs;
                l.xs = e.x;
                l.y = j->Bd + j->ad_off[r0];
                l.w = j->WL;
                l.flags = hs::kElimTrans | hs::kElimStrict;
                l.dfin = nullptr;
                es.push_back(l);
            }
        }
        hs::PairStep* d_ps = tmp.upload(ps, s);
        hs::launch_pair_table(d_ps, (int64_t)ps.size(), j->d_err, s);
        j->d_kept = true;
    }
    // components: the steps of each, in order (a component's steps are those
    // with the same elimination-tree root)
    std::vector<std::vector<std::pair<size_t, int64_t>>> comps;
    for (size_t q = 0; q < jobs.size(); ++q) {
        SetupJob* j = jobs[q];
        const hs::Symbolic& sy = j->P->plan.sym;
        std::vector<int64_t> root(j->nb);
        for (int64_t k = j->nb - 1; k >= 0; --k) root[k] = sy.parent[k] < 0 ? k : root[sy.parent[k]];
        std::unordered_map<int64_t, size_t> cid;
        for (int64_t k = 0; k < j->nb; ++k) {
            auto it = cid.find(root[k]);
            if (it == cid.end()) {
                it = cid.emplace(root[k], comps.size()).first;
                comps.emplace_back();
            }
            comps[it->second].push_back({q, k});
        }
    }
    // the look-ahead: flags, previous entries and the maps of S_k into S_p
    for (const auto& c : comps) {
        for (size_t i = 1; i < c.size(); ++i) {
            const size_t q = c[i].first;
            SetupJob* j = jobs[q];
            if (j->nonsym) continue;
            const int64_t kp = c[i - 1].second, k = c[i].second;
            const hs::Symbolic& sy = j->P->plan.sym;
            const int64_t p0 = sy.rowptr[kp], p1 = sy.rowptr[kp + 1];
            if (p1 == p0 || sy.cols[p0] != k) continue;
            // only where the factor tile stages its look-ahead operands in
            // LDS (b_k <= 32, b_p <= 64): for larger blocks the update's
            // global-memory round trips cost more than the Schur launch
            if (j->P->bsize[k] > 32 || j->P->bsize[kp] > 64) continue;
            const int32_t ep = sidx[q][kp], ek = sidx[q][k];
            es[ek].flags |= hs::kElimLook;
            es[ek].prev = ep;
            es[ep].flags |= hs::kElimSkip0;
            // each block of S_k: its first column in kp's panel (S_kp sorted; -1 if absent)
            const int64_t r0 = sy.rowptr[k], r1 = sy.rowptr[k + 1];
            int64_t e2 = p0;
            for (int64_t e = r0; e < r1; ++e) {
                while (e2 < p1 && sy.cols[e2] < sy.cols[e]) ++e2;
                lamap_h[q][e] = (e2 < p1 && sy.cols[e2] == sy.cols[e]) ? j->pcol[p0 + kp + (e2 - p0)] : -1;
            }
        }
    }
    for (size_t q = 0; q < jobs.size(); ++q)
        hip_check(hipMemcpyAsync(lamap_d[q], lamap_h[q].data(), sizeof(int32_t) * lamap_h[q].size(),
                                 hipMemcpyHostToDevice, s), "upload lamap");
    // the launch groups of each component, then launch g = every component's g-th group
    auto add_f = [&](std::vector<hs::ElimTile>& out, size_t q, int64_t k) {
        const int32_t e0 = sidx[q][k];
        const int32_t nent = jobs[q]->nonsym && jobs[q]->panel_m[k] > 0 ? 2 : 1;
        const int32_t nt = std::max<int32_t>(1, (jobs[q]->panel_m[k] + 63) / 64);
        for (int32_t t = 0; t < nent; ++t)
            for (int32_t i = 0; i < nt; ++i) out.push_back(hs::ElimTile{e0 + t, (int16_t)i, -1});
    };
    auto add_s = [&](std::vector<hs::ElimTile>& out, size_t q, int64_t k) {
        SetupJob* j = jobs[q];
        const int32_t e0 = sidx[q][k];
        const int32_t nent = j->nonsym && j->panel_m[k] > 0 ? 2 : 1;
        for (int32_t t = 0; t < nent; ++t)
            for (int64_t i = j->tile_ptr[k]; i < j->tile_ptr[k + 1]; ++i)
                out.push_back(hs::ElimTile{e0 + t, j->tiles[i].first, j->tiles[i].second});
    };
    std::vector<std::vector<hs::ElimTile>> groups;
    for (const auto& c : comps) {
        size_t g = 0;
        auto at = [&](size_t gi) -> std::vector<hs::ElimTile>& {
            if (groups.size() <= gi) groups.resize(gi + 1);
            return groups[gi];
        };
        add_f(at(g++), c[0].first, c[0].second);
        for (size_t i = 0; i < c.size(); ++i) {
            const size_t q = c[i].first;
            const bool next = i + 1 < c.size();
            if (next && (es[sidx[q][c[i + 1].second]].flags & hs::kElimLook)) {
                auto& grp = at(g++);
                add_f(grp, q, c[i + 1].second);
                add_s(grp, q, c[i].second);
            } else {
                add_s(at(g++), q, c[i].second);
                if (next) add_f(at(g++), q, c[i + 1].second);
            }
        }
    }
    std::vector<int64_t> gp(groups.size() + 1, 0);
    std::vector<hs::ElimTile> items;
    for (size_t g = 0; g < groups.size(); ++g) {
        items.insert(items.end(), groups[g].begin(), groups[g].end());
        gp[g + 1] = (int64_t)items.size();
    }
    const hs::ElimStep* d_es = tmp.upload(es, s);
    const hs::ElimTile* d_items = tmp.upload(items, s);
    hs_context* ctx = jobs.front()->ctx;
    const bool fp32 = jobs.front()->opts->precision == HS_PREC_MIXED;
    timed(ctx, HS_KT_ELIM, s, [&] {
        for (size_t g = 0; g < groups.size(); ++g) {
            bool has_f = false;
            for (int64_t i = gp[g]; i < gp[g + 1] && !has_f; ++i) has_f = items[i].tj < 0;
            timed(ctx, has_f ? HS_KT_FACTOR : HS_KT_SCHUR, s,
                  [&] { hs::launch_elim_items(d_es, d_items + gp[g], gp[g + 1] - gp[g], fp32, s); });
        }
    });
    hip_check(hipGetLastError(), "elimination launches");
    hip_check(hipStreamSynchronize(s), "stream sync");
}

}  // namespace

extern "C" {

// ---- preconditioner setup ---------------------------------------------------------

int32_t hs_precond_setup(hs_context* ctx, const hs_hmatrix* H, const hs_precond_opts* opts, hs_precond** out) {
    if (!out) { g_last_error = "out is NULL"; return HS_EINVAL; }
    return hs_precond_setup_many(ctx, 1, &H, opts, out);
}

int32_t hs_precond_setup_many(hs_context* ctx, int64_t count, const hs_hmatrix* const* Hs, const hs_precond_opts* opts,
                              hs_precond** out) {
    try {
        if (!out) fail(HS_EINVAL, "out is NULL");
        if (count < 1) fail(HS_EINVAL, "count must be >= 1");
        for (int64_t g = 0; g < count; ++g) out[g] = nullptr;
        if (!Hs) fail(HS_EINVAL, "NULL argument");
        for (int64_t g = 0; g < count; ++g) {
            const hs_hmatrix* H = Hs[g];
        if (!ctx || !H || !opts) fail(HS_EINVAL, "NULL argument");
            if (opts->ordering < 0 || opts->ordering > 4) fail(HS_EINVAL, "unknown ordering");
            if (!(opts->fill_tol >= 0.0)) fail(HS_EINVAL, "fill_tol must be >= 0");
            if (opts->precision != HS_PREC_FP64 && opts->precision != HS_PREC_MIXED) fail(HS_EINVAL, "unsupported precision");
            if (opts->kind != HS_PC_SCHUR && opts->kind != HS_PC_BLOCK_JACOBI && opts->kind != HS_PC_SCHUR_NONSYM &&
                opts->kind != HS_PC_SCHUR_LOWRANK)
                fail(HS_EINVAL, "unknown preconditioner kind");
            if (opts->kind == HS_PC_SCHUR_LOWRANK && opts->precision != HS_PREC_FP64)
                fail(HS_EINVAL, "the low-rank setup arithmetic is FP64 only");
            if (opts->kind == HS_PC_BLOCK_JACOBI && opts->precision != HS_PREC_FP64)
                fail(HS_EINVAL, "the block-Jacobi comparator is FP64 only");
            if (opts->sweep_chunk < 0 || opts->sweep_chunk > hs::kMaxChunk) fail(HS_EINVAL, "sweep_chunk must be in [0, 384]");
            const int32_t chunk_lim = opts->sweep_chunk > 0 ? opts->sweep_chunk : hs::kMaxChunk;
            if (opts->sweep_fold_cols != 0 && (opts->sweep_fold_cols < chunk_lim || opts->sweep_fold_cols > hs::kFoldCols))
                fail(HS_EINVAL, "sweep_fold_cols must be 0 or in [chunk size, 3072]");
            set_device(ctx);
            // the sweeps keep their row workers resident for a whole launch
            // and need others beside them
            if (hs::sweep_capacity(ctx->device) < hs::kRowWorkers * hs::kRowSets + 32)
                fail(HS_ENODEVICE, "too few resident workgroups for the preconditioner sweeps");
            if (H->plan.part.n_near() == 0) fail(HS_EINVAL, "empty H-matrix");
        }
        std::vector<std::unique_ptr<SetupJob>> jobs;
        std::vector<SetupJob*> jp;
        for (int64_t g = 0; g < count; ++g) {
            auto j = std::make_unique<SetupJob>();
            j->ctx = ctx;
            j->H = Hs[g];
            j->opts = opts;
            j->s = ctx->stream;
            j->chunk_lim = opts->sweep_chunk > 0 ? opts->sweep_chunk : hs::kMaxChunk;
            j->fold_cols = opts->sweep_fold_cols > 0 ? opts->sweep_fold_cols : hs::kFoldCols;
            j->prepare();
            jp.push_back(j.get());
            jobs.push_back(std::move(j));
        }
        if (opts->kind == HS_PC_SCHUR_LOWRANK) {
            // one geometry at a time: each step's ranks come back to the host
            for (auto& j : jobs) j->eliminate_lowrank();
        } else {
            eliminate(jp, ctx->stream);
        }
        for (auto& j : jobs) j->finish();
        for (int64_t g = 0; g < count; ++g) out[g] = jobs[g]->P.release();
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return HS_ENOMEM;
    }
}

int32_t hs_precond_tune(hs_context* ctx, const hs_hmatrix* H, const hs_precond_opts* opts, int32_t nrhs, int32_t reps,
                        hs_precond_opts* best, double* times_ms, int32_t* ncand) {
    try {
        if (!ctx || !H || !opts || !best) fail(HS_EINVAL, "NULL argument");
        if (nrhs < 1 || reps < 1) fail(HS_EINVAL, "nrhs and reps must be >= 1");
        if (opts->kind != HS_PC_SCHUR) fail(HS_EINVAL, "the layouts belong to the Schur preconditioner");
        // the candidate grid: chunk sizes x folded-range widths (width >= chunk)
        static const int32_t chunks[] = {384, 256, 192};
        static const int32_t folds[] = {3072, 2048, 1536};
        set_device(ctx);
        hipStream_t s = ctx->stream;
        const int64_t n = H->n;
        Owned w;
        w.mem = ctx->mem;
        cd* v = w.get<cd>((size_t)n * nrhs);
        cd* z = w.get<cd>((size_t)n * nrhs);
        std::vector<cd> ones((size_t)n * nrhs);
        for (auto& e : ones) { e.x = 1.0; e.y = 0.0; }
        hip_check(hipMemcpyAsync(v, ones.data(), sizeof(cd) * ones.size(), hipMemcpyHostToDevice, s), "H2D");
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        double best_ms = 0.0;
        int32_t k = 0;
        for (int32_t c : chunks) {
            for (int32_t f : folds) {
                if (f < c) continue;
                hs_precond_opts o = *opts;
                o.sweep_chunk = c;
                o.sweep_fold_cols = f;
                hs_precond* P = nullptr;
                const int32_t rc = hs_precond_setup(ctx, H, &o, &P);
                if (rc != HS_OK) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return rc;
                }
                std::unique_ptr<hs_precond, void (*)(hs_precond*)> pg(P, hs_precond_destroy);
                SweepWs sw = make_sweep_ws(w, P, nrhs, s, ctx);
                apply_tree(ctx, P, v, z, nrhs, sw, s, kAllCols);   // warm-up
                hip_check(hipEventRecord(e0, s), "hipEventRecord");
                for (int32_t r = 0; r < reps; ++r) apply_tree(ctx, P, v, z, nrhs, sw, s, kAllCols);
                hip_check(hipEventRecord(e1, s), "hipEventRecord");
                hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                check_sweep_flag(sw, s);
                float ms = 0.0f;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                const double avg = (double)ms / reps;
                if (times_ms) times_ms[k] = avg;
                if (k == 0 || avg < best_ms) {
                    best_ms = avg;
                    *best = o;
                }
                ++k;
            }
        }
        if (ncand) *ncand = k;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_query_precond(const hs_precond* P, hs_info* info) {
    if (!P || !info) { g_last_error = "NULL argument"; return HS_EINVAL; }
    fill_info_plan(P->plan, info);
    info->n_lowrank = P->n_lowrank;
    info->bytes_alpha = P->alpha_elems * 16;
    info->bytes_d = P->d_elems * 16;
    info->flops_fill = P->flops_fill;
    if (P->flops_factored > 0) info->flops_setup = P->flops_factored;
    info->bytes_device = P->own.bytes;
    return HS_OK;
}

void hs_precond_destroy(hs_precond* P) { delete P; }

int32_t hs_precond_export(const hs_precond* P, int32_t what, void* dst, int64_t cap, int64_t* needed) {
    try {
        if (!P) fail(HS_EINVAL, "P is NULL");
        if (what >= HS_X_PERM && what <= HS_X_ORIG) return export_plan(P->plan, what, dst, cap, needed);
        hip_check(hipSetDevice(P->own.mem.device), "hipSetDevice");
        hip_check(hipDeviceSynchronize(), "device sync");
        switch (what) {
            case HS_P_D: return copy_out(P->d_D, P->d_elems * 16, dst, cap, needed, nullptr);
            case HS_P_ALPHA_KIND: {
                std::vector<int64_t> v(P->a_rank.begin(), P->a_rank.end());
                return copy_host(v, dst, cap, needed);
            }
            case HS_P_ALPHA_OFF: {
                std::vector<int64_t> v = P->a_off;
                v.push_back(P->alpha_elems);
                return copy_host(v, dst, cap, needed);
            }
            case HS_P_ALPHA: return copy_out(P->d_alpha, P->alpha_elems * 16, dst, cap, needed, nullptr);
            case HS_P_ALPHA_LEFT:
                if (!P->d_alpha_left) fail(HS_EINVAL, "only a non-symmetric setup keeps the left coefficients");
                return copy_out(P->d_alpha_left, P->alpha_left_elems * 16, dst, cap, needed, nullptr);
            default: fail(HS_EINVAL, "unknown export code");
        }
    } catch (const Error& e) {
        return set_error(e);
    }
}

// ---- operator applications -------------------------------------------------------

int32_t hs_matvec(hs_context* ctx, const hs_hmatrix* H, const void* x, void* y, int64_t nrhs) {
    try {
        if (!ctx || !H || !x || !y) fail(HS_EINVAL, "NULL argument");
        if (nrhs < 1) fail(HS_EINVAL, "nrhs must be >= 1");
        H->join_far();
        set_device(ctx);
        hipStream_t s = ctx->stream;
        Owned w;
        w.mem = ctx->mem;
        const int64_t n = H->n;
        cd* xt = w.get<cd>(n * nrhs);
        cd* yt = w.get<cd>(n * nrhs);
        cd* slots = w.get<cd>(H->slot_total * nrhs);
        hs::launch_permute(static_cast<const cd*>(x), xt, H->d_perm, n, nrhs, true, s);
        matvec_tree(ctx, H, xt, yt, (int)nrhs, slots, s, kAllCols);
        hs::launch_permute(yt, static_cast<cd*>(y), H->d_perm, n, nrhs, false, s);
        hip_check(hipGetLastError(), "matvec launches");
        hip_check(hipStreamSynchronize(s), "stream sync");
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_matvec_noalloc(hs_context* ctx, const hs_hmatrix* H, const void* x, void* y, int64_t nrhs,
                          int64_t* scratch_needed) {
    try {
        if (!ctx || !H || !x || !y) fail(HS_EINVAL, "NULL argument");
        if (nrhs < 1) fail(HS_EINVAL, "nrhs must be >= 1");
        H->join_far();   // a no-op once the far field is in (no allocation)
        auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
        const int64_t n = H->n;
        const size_t vbytes = up(sizeof(cd) * (size_t)n * (size_t)nrhs);
        const size_t sbytes = up(sizeof(cd) * (size_t)H->slot_total * (size_t)nrhs);
        const size_t need = 2 * vbytes + sbytes;
        if (scratch_needed) *scratch_needed = (int64_t)need;
        if (need > kNoAllocScratchBytes)
            fail(HS_EINVAL, "hs_matvec_noalloc needs " + std::to_string(need) + " bytes of scratch, more than its " +
                                std::to_string(kNoAllocScratchBytes) + "-byte device array");
        unsigned char* base = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_scratch.mu);
            base = static_cast<unsigned char*>(g_scratch.ptr[ctx->device]);
        }
        if (!base) fail(HS_EHIP, "the scratch address of this device is unknown");
        set_device(ctx);
        hipStream_t s = ctx->stream;
        cd* xt = reinterpret_cast<cd*>(base);
        cd* yt = reinterpret_cast<cd*>(base + vbytes);
        cd* slots = reinterpret_cast<cd*>(base + 2 * vbytes);
        // near and far kernels one after the other on the context's stream
        // (no auxiliary stream or events), each writing its own slots; the
        // gather adds them; every scratch word read was written in this call
        hs::launch_permute(static_cast<const cd*>(x), xt, H->d_perm, n, nrhs, true, s);
        hs::launch_near_mv(kAllCols, H->d_near_tasks, H->d_near_slot, (int64_t)H->near_tasks.size(), H->d_near, xt, n,
                           (int)nrhs, slots, s);
        hs::launch_far_mv(kAllCols, H->d_mv_geom, H->d_mv_rank, H->d_mv_ptr, H->d_mv_slot, H->n_far_wg,
                          (int64_t)H->far_geom.size(), xt, n, (int)nrhs, slots, s);
        hs::launch_gather(kAllCols, H->d_leaf_off, H->d_gptr, H->d_gent, H->nb, slots, n, (int)nrhs, yt, s);
        hs::launch_permute(yt, static_cast<cd*>(y), H->d_perm, n, nrhs, false, s);
        hip_check(hipGetLastError(), "matvec launches");
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_precond_apply(hs_context* ctx, const hs_precond* P, const void* v, void* z, int64_t nrhs) {
    try {
        if (!ctx || !P || !v || !z) fail(HS_EINVAL, "NULL argument");
        if (nrhs < 1) fail(HS_EINVAL, "nrhs must be >= 1");
        set_device(ctx);
        hipStream_t s = ctx->stream;
        Owned w;
        w.mem = ctx->mem;
        const int64_t n = P->H->n;
        cd* vt = w.get<cd>(n * nrhs);
        cd* zt = w.get<cd>(n * nrhs);
        SweepWs sw = make_sweep_ws(w, P, (int)nrhs, s, ctx);
        hs::launch_permute(static_cast<const cd*>(v), vt, P->H->d_perm, n, nrhs, true, s);
        apply_tree(ctx, P, vt, zt, (int)nrhs, sw, s, kAllCols);
        hs::launch_permute(zt, static_cast<cd*>(z), P->H->d_perm, n, nrhs, false, s);
        hip_check(hipGetLastError(), "apply launches");
        check_sweep_flag(sw, s);
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

// ---- solve -------------------------------------------------------------------------

}  // extern "C"

namespace {

using ApplyFn = std::function<void(const cd* in, cd* out, const hs::ColMask& mk)>;

// Inner polls one poll behind: at each poll point the column states (and the
// sweeps' error flag) are copied into pinned host memory behind an event,
// and the host reads the copy of the previous poll point, whose work has
// long finished, instead of draining the stream. The launches for the next
// group of steps are therefore queued before the GPU runs out of work.
// Steps taken after a column stopped skip it (the kernels read its state),
// so the lag costs at most one group of empty steps when all have stopped.
struct PollRing {
    hs::ColState* h = nullptr;   // pinned: 2 slots of ns states
    int* err = nullptr;          // pinned: 2 flags
    hipEvent_t ev[2] = {nullptr, nullptr};
    int ns = 0, next = 0, pending = -1;
    explicit PollRing(int ns_) : ns(ns_) {
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&h), sizeof(hs::ColState) * 2 * ns, hipHostMallocDefault),
                  "hipHostMalloc");
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&err), sizeof(int) * 2, hipHostMallocDefault),
                  "hipHostMalloc");
        for (auto& e : ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
    }
    ~PollRing() {
        if (pending >= 0) (void)hipEventSynchronize(ev[pending]);   // a copy may still land in h / err
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (h) (void)hipHostFree(h);
        if (err) (void)hipHostFree(err);
    }
    PollRing(const PollRing&) = delete;
    PollRing& operator=(const PollRing&) = delete;
    // Queue this poll point's copies; true when the previous poll point saw
    // no column still stepping.
    bool poll(const hs::ColState* d_st, const int* sweep_err, hipStream_t s) {
        const int k = next;
        err[k] = 0;
        hip_check(hipMemcpyAsync(h + (size_t)k * ns, d_st, sizeof(hs::ColState) * ns, hipMemcpyDeviceToHost, s), "D2H");
        if (sweep_err) hip_check(hipMemcpyAsync(err + k, sweep_err, sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipEventRecord(ev[k], s), "hipEventRecord");
        next ^= 1;
        const int q = pending;
        pending = k;
        if (q < 0) return false;
        hip_check(hipEventSynchronize(ev[q]), "hipEventSynchronize");
        if (err[q] != 0)
            fail(HS_ETIMEOUT, "a device-side wait of the preconditioner sweeps exceeded the context's wait limit");
        bool any = false;
        for (int c = 0; c < ns; ++c) any |= h[(size_t)q * ns + c].active != 0;
        return !any;
    }
    // Start of a cycle: the copy still pending (if any) lands first.
    void reset() {
        if (pending >= 0) hip_check(hipEventSynchronize(ev[pending]), "hipEventSynchronize");
        pending = -1;
    }
};

// Workspace of a multi-column GMRES(m) (or flexible GMRES(m): Z keeps the
// preconditioned basis) on tree-order vectors.
struct GmresWs {
    int64_t n = 0, vstride = 0, ldh = 0;
    int ns = 0, m = 0, nchunk = 0;
    cd *r, *wv, *tmp, *V, *Z, *Hh, *snv, *g, *y, *partial;
    double *csv, *npart;
    hs::ColState* st;
    std::shared_ptr<PollRing> ring;   // created at the first solve on this workspace
    void alloc(Owned& w, int64_t n_, int ns_, int m_, bool flexible) {
        n = n_;
        ns = ns_;
        m = m_;
        nchunk = hs::gmres_nchunk(n);
        vstride = n * ns;
        ldh = (int64_t)(m + 1) * m;
        r = w.get<cd>(n * ns);
        wv = w.get<cd>(n * ns);
        tmp = w.get<cd>(n * ns);
        V = w.get<cd>((size_t)(m + 1) * vstride);
        Z = flexible ? w.get<cd>((size_t)m * vstride) : nullptr;
        Hh = w.get<cd>((size_t)ldh * ns);
        csv = w.get<double>((size_t)m * ns);
        snv = w.get<cd>((size_t)m * ns);
        g = w.get<cd>((size_t)(m + 1) * ns);
        y = w.get<cd>((size_t)m * ns);
        partial = w.get<cd>((size_t)nchunk * (m + 1) * ns);
        npart = w.get<double>((size_t)nchunk * ns);
        st = w.get<hs::ColState>(ns);
    }
};

// Restart cycles of right-preconditioned GMRES(m) from x = 0 (x must hold
// zeros), with the column states already initialised in G.st. Plain: the
// preconditioned vector only feeds the matvec and x += P^-1 (V y).
// Flexible: z_j = precond(v_j) is kept and x += Z y. single: one cycle and
// no true-residual pass (inner solves). Otherwise cycles run until every
// column is done; inside a cycle only the columns still stepping are
// computed, at its end those that stepped.
// Column states to the host at a poll, with the sweeps' error flag (bounded
// waits) read in the same synchronisation.
std::vector<hs::ColState> poll_states(const GmresWs& G, const int* sweep_err, hipStream_t s) {
    std::vector<hs::ColState> h(G.ns);
    int err = 0;
    hip_check(hipMemcpyAsync(h.data(), G.st, sizeof(hs::ColState) * G.ns, hipMemcpyDeviceToHost, s), "D2H");
    if (sweep_err) hip_check(hipMemcpyAsync(&err, sweep_err, sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "stream sync");
    if (err != 0)
        fail(HS_ETIMEOUT, "a device-side wait of the preconditioner sweeps exceeded the context's wait limit");
    return h;
}

// resid (optional) replaces matvec for the true residual at each cycle end:
// with the FP64 operator there, a cycle built on complex64 copies becomes one
// step of iterative refinement.
void gmres_run(GmresWs& G, hipStream_t s, const cd* b, cd* x, const ApplyFn& matvec, const ApplyFn& precond,
               bool flexible, bool single, int poll, const int* sweep_err, const ApplyFn* resid = nullptr) {
    const int64_t n = G.n, vs = G.vstride;
    const int ns = G.ns, m = G.m;
    const hs::ColMask active{G.st, 1, 0}, stepped{G.st, 2, 0};
    hip_check(hipMemsetAsync(G.Hh, 0, sizeof(cd) * G.ldh * ns, s), "memset");
    hs::launch_col_norms(b, n, ns, G.npart, G.nchunk, s);
    hs::launch_cycle_start(b, G.V, n, G.g, m, G.npart, G.nchunk, G.st, n, ns, true, s);
    if (!G.ring || G.ring->ns != ns) G.ring = std::make_shared<PollRing>(ns);
    PollRing& ring = *G.ring;
    for (;;) {
        ring.reset();
        for (int j = 0; j < m; ++j) {
            cd* zj = flexible ? G.Z + j * vs : G.tmp;
            precond(G.V + j * vs, zj, active);
            matvec(zj, G.wv, active);
            hs::launch_dots(G.V, n, vs, j + 1, G.wv, n, ns, G.st, G.partial, G.nchunk, s);
            hs::launch_basis_update(G.V, n, vs, j + 1, G.partial, G.nchunk, G.wv, n, ns, G.st, G.Hh, G.ldh, m + 1, j,
                                    false, nullptr, s);
            hs::launch_dots(G.V, n, vs, j + 1, G.wv, n, ns, G.st, G.partial, G.nchunk, s);
            hs::launch_basis_update(G.V, n, vs, j + 1, G.partial, G.nchunk, G.wv, n, ns, G.st, G.Hh, G.ldh, m + 1, j,
                                    true, G.npart, s);
            hs::launch_givens_scale(G.Hh, G.ldh, m, j, G.csv, G.snv, G.g, G.npart, G.nchunk, G.st, ns, G.wv,
                                    G.V + (j + 1) * vs, n, n, s);
            if ((j + 1) % poll == 0 && j + 1 < m) {
                hip_check(hipGetLastError(), "inner launches");
                if (ring.poll(G.st, sweep_err, s)) break;
            }
        }
        hs::launch_lsq(G.Hh, G.ldh, m, G.g, G.y, G.st, ns, s);
        if (flexible) {
            hs::launch_combine(G.Z, n, vs, G.y, m, G.tmp, n, ns, G.st, s);
            hs::launch_axpy_x(x, G.tmp, n, ns, G.st, s);
        } else {
            hs::launch_combine(G.V, n, vs, G.y, m, G.tmp, n, ns, G.st, s);
            precond(G.tmp, G.wv, stepped);
            hs::launch_axpy_x(x, G.wv, n, ns, G.st, s);
        }
        if (single) break;
        (resid ? *resid : matvec)(x, G.tmp, stepped);
        hs::launch_residual(b, G.tmp, G.r, n, ns, G.npart, G.nchunk, s);
        hs::launch_cycle_end(G.npart, G.nchunk, G.st, ns, s);
        hip_check(hipGetLastError(), "cycle launches");
        std::vector<hs::ColState> cur = poll_states(G, sweep_err, s);
        bool all_done = true;
        for (auto& c : cur) all_done &= c.done != 0;
        if (all_done) break;
        hip_check(hipMemsetAsync(G.Hh, 0, sizeof(cd) * G.ldh * ns, s), "memset");
        hs::launch_cycle_start(G.r, G.V, n, G.g, m, G.npart, G.nchunk, G.st, n, ns, false, s);
    }
}


// ---- coupled block GMRES (comparator) -----------------------------------------------

typedef std::complex<double> zc;

void blas_check(rocblas_status st, const char* what) {
    if (st != rocblas_status_success) fail(HS_EHIP, std::string(what) + ": rocBLAS status " + std::to_string((int)st));
}

rocblas_handle ctx_blas(hs_context* ctx) {
    if (!ctx->blas) blas_check(rocblas_create_handle(&ctx->blas), "rocblas_create_handle");
    blas_check(rocblas_set_stream(ctx->blas, ctx->stream), "rocblas_set_stream");
    blas_check(rocblas_set_pointer_mode(ctx->blas, rocblas_pointer_mode_host), "rocblas_set_pointer_mode");
    return ctx->blas;
}

const rocblas_double_complex* rz(const zc* p) { return reinterpret_cast<const rocblas_double_complex*>(p); }
const rocblas_double_complex* rz(const cd* p) { return reinterpret_cast<const rocblas_double_complex*>(p); }
rocblas_double_complex* rz(cd* p) { return reinterpret_cast<rocblas_double_complex*>(p); }

// Cholesky G = C^H C of an s x s Hermitian matrix (column-major); false if a
// pivot is not positive (the columns are dependent).
bool chol_upper(const std::vector<zc>& G, int s, std::vector<zc>& C) {
    C.assign((size_t)s * s, zc(0.0, 0.0));
    for (int j = 0; j < s; ++j) {
        for (int i = 0; i <= j; ++i) {
            zc sum = G[(size_t)i + (size_t)j * s];
            for (int l = 0; l < i; ++l) sum -= std::conj(C[(size_t)l + (size_t)i * s]) * C[(size_t)l + (size_t)j * s];
            if (i == j) {
                const double d = sum.real();
                if (!(d > 0.0)) return false;
                C[(size_t)j + (size_t)j * s] = zc(std::sqrt(d), 0.0);
            } else {
                C[(size_t)i + (size_t)j * s] = sum / C[(size_t)i + (size_t)i * s];
            }
        }
    }
    return true;
}

// In place W (n x s, device) = Q R by Cholesky QR applied twice; R (host,
// s x s upper, column-major) = C2 C1. False on dependent columns.
bool cholqr2(rocblas_handle hb, cd* W, int64_t n, int s, cd* d_g, std::vector<zc>& R, hipStream_t st) {
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    std::vector<zc> G((size_t)s * s), C, Rt((size_t)s * s, zc(0.0, 0.0));
    for (int i = 0; i < s; ++i) Rt[(size_t)i + (size_t)i * s] = zc(1.0, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
        blas_check(rocblas_zgemm(hb, rocblas_operation_conjugate_transpose, rocblas_operation_none, s, s, (int)n, &one,
                                 rz(W), (int)n, rz(W), (int)n, &zero, rz(d_g), s), "zgemm (W^H W)");
        hip_check(hipMemcpyAsync(G.data(), d_g, sizeof(zc) * s * s, hipMemcpyDeviceToHost, st), "D2H");
        hip_check(hipStreamSynchronize(st), "stream sync");
        if (!chol_upper(G, s, C)) return false;
        hip_check(hipMemcpyAsync(d_g, C.data(), sizeof(zc) * s * s, hipMemcpyHostToDevice, st), "H2D");
        blas_check(rocblas_ztrsm(hb, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                 rocblas_diagonal_non_unit, (int)n, s, &one, rz(d_g), s, rz(W), (int)n),
                   "ztrsm (W C^-1)");
        std::vector<zc> nr((size_t)s * s, zc(0.0, 0.0));   // C Rt
        for (int j = 0; j < s; ++j)
            for (int i = 0; i <= j; ++i) {
                zc acc(0.0, 0.0);
                for (int l = i; l <= j; ++l) acc += C[(size_t)i + (size_t)l * s] * Rt[(size_t)l + (size_t)j * s];
                nr[(size_t)i + (size_t)j * s] = acc;
            }
        Rt.swap(nr);
    }
    R.swap(Rt);
    return true;
}

// min || rhs - H Y ||_F column by column for H (M x K, column-major, M > K)
// by complex Householder QR; returns Y (K x ns) and each column's residual norm.
void block_ls(std::vector<zc> H, int M, int K, std::vector<zc> rhs, int ns, std::vector<zc>& Y,
              std::vector<double>& res) {
    for (int c = 0; c < K; ++c) {
        double nrm = 0.0;
        for (int i = c; i < M; ++i) nrm += std::norm(H[(size_t)i + (size_t)c * M]);
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const zc a = H[(size_t)c + (size_t)c * M];
        const zc ph = std::abs(a) > 0.0 ? a / std::abs(a) : zc(1.0, 0.0);
        const zc alpha = -ph * nrm;
        std::vector<zc> v((size_t)(M - c));
        for (int i = c; i < M; ++i) v[(size_t)(i - c)] = H[(size_t)i + (size_t)c * M];
        v[0] -= alpha;
        double vn = 0.0;
        for (auto& e : v) vn += std::norm(e);
        if (vn == 0.0) continue;
        auto reflect = [&](zc* col) {
            zc d(0.0, 0.0);
            for (int i = c; i < M; ++i) d += std::conj(v[(size_t)(i - c)]) * col[i];
            d *= 2.0 / vn;
            for (int i = c; i < M; ++i) col[i] -= d * v[(size_t)(i - c)];
        };
        for (int j = c; j < K; ++j) reflect(&H[(size_t)j * M]);
        for (int j = 0; j < ns; ++j) reflect(&rhs[(size_t)j * M]);
    }
    Y.assign((size_t)K * ns, zc(0.0, 0.0));
    res.assign(ns, 0.0);
    for (int j = 0; j < ns; ++j) {
        for (int i = K - 1; i >= 0; --i) {
            zc sum = rhs[(size_t)i + (size_t)j * M];
            for (int l = i + 1; l < K; ++l) sum -= H[(size_t)i + (size_t)l * M] * Y[(size_t)l + (size_t)j * K];
            const zc d = H[(size_t)i + (size_t)i * M];
            Y[(size_t)i + (size_t)j * K] = std::abs(d) > 0.0 ? sum / d : zc(0.0, 0.0);
        }
        double r = 0.0;
        for (int i = K; i < M; ++i) r += std::norm(rhs[(size_t)i + (size_t)j * M]);
        res[j] = std::sqrt(r);
    }
}

// Coupled block GMRES(m), right-preconditioned: one Krylov space for the
// nrhs columns (see hschur.h). Steps are block steps.
int32_t solve_block(hs_context* ctx, const hs_hmatrix* H, const hs_precond* P, const void* b, void* x, int64_t nrhs,
                    const hs_solve_opts* opts, hs_solve_stats* stats) {
    if (opts->use_x0) fail(HS_EINVAL, "use_x0 is supported by HS_SOLVE_GMRES only");
    const int m = opts->restart;
    if (m < 1 || m > hs::kMaxRankCap) fail(HS_EINVAL, "restart must be in [1, 256]");
    if (!(opts->tol >= 0.0)) fail(HS_EINVAL, "tol must be >= 0");
    if (nrhs > 256) fail(HS_EINVAL, "block GMRES takes at most 256 columns");
    const int budget = opts->fixed_iters > 0 ? opts->fixed_iters : (opts->max_iters > 0 ? opts->max_iters : 5000);
    const bool fixed = opts->fixed_iters > 0;
    set_device(ctx);
    hipStream_t st = ctx->stream;
    rocblas_handle hb = ctx_blas(ctx);
    const int64_t n = H->n;
    const int ns = (int)nrhs;
    const int64_t blk = n * ns;
    Owned w;
    w.mem = ctx->mem;
    cd* bt = w.get<cd>(blk);
    cd* xt = w.get<cd>(blk);
    cd* V = w.get<cd>((size_t)(m + 1) * blk);
    cd* Wt = w.get<cd>(blk);
    cd* tmp = w.get<cd>(blk);
    cd* d_h = w.get<cd>((size_t)(m + 1) * ns * ns);
    cd* d_g = w.get<cd>((size_t)ns * ns);
    cd* d_y = w.get<cd>((size_t)m * ns * ns);
    cd* slots = w.get<cd>((size_t)H->slot_total * ns);
    const int nchunk = hs::gmres_nchunk(n);
    double* npart = w.get<double>((size_t)nchunk * ns);
    SweepWs sw;
    if (P) sw = make_sweep_ws(w, P, ns, st, ctx);
    hs::launch_permute(static_cast<const cd*>(b), bt, H->d_perm, n, ns, true, st);
    hip_check(hipMemsetAsync(xt, 0, sizeof(cd) * blk, st), "memset");
    auto col_norms = [&](const cd* v) {
        hs::launch_col_norms(v, n, ns, npart, nchunk, st);
        std::vector<double> pp = download(npart, (size_t)nchunk * ns, st);
        std::vector<double> out(ns, 0.0);
        for (int c = 0; c < ns; ++c) {
            for (int ch = 0; ch < nchunk; ++ch) out[c] += pp[(size_t)ch * ns + c];
            out[c] = std::sqrt(out[c]);
        }
        return out;
    };
    auto precond = [&](const cd* in, cd* out) {
        if (P) apply_tree(ctx, P, in, out, ns, sw, st, kAllCols);
        else hip_check(hipMemcpyAsync(out, in, sizeof(cd) * blk, hipMemcpyDeviceToDevice, st), "D2D");
    };
    const std::vector<double> bn = col_norms(bt);
    const rocblas_double_complex one{1.0, 0.0}, mone{-1.0, 0.0}, zero{0.0, 0.0};
    int steps = 0;
    std::vector<double> rel(ns, 1.0);
    bool first = true;
    for (;;) {
        // R = B - Z X into V_0, then V_0 S = R
        if (first) {
            hip_check(hipMemcpyAsync(V, bt, sizeof(cd) * blk, hipMemcpyDeviceToDevice, st), "D2D");
        } else {
            matvec_tree(ctx, H, xt, tmp, ns, slots, st, kAllCols);
            hs::launch_residual(bt, tmp, V, n, ns, npart, nchunk, st);
        }
        first = false;
        std::vector<zc> S;
        if (!cholqr2(hb, V, n, ns, d_g, S, st)) break;   // dependent residual columns
        std::vector<zc> Hb((size_t)(m + 1) * ns * m * ns, zc(0.0, 0.0));
        const int M0 = (m + 1) * ns;
        std::vector<zc> Y;
        int k = 0;
        while (k < m && steps < budget) {
            cd* Vk = V + (size_t)k * blk;
            cd* Vn = V + (size_t)(k + 1) * blk;
            precond(Vk, Wt);
            matvec_tree(ctx, H, Wt, Vn, ns, slots, st, kAllCols);
            const int kc = (k + 1) * ns;
            std::vector<zc> h((size_t)kc * ns, zc(0.0, 0.0)), h2((size_t)kc * ns);
            for (int pass = 0; pass < 2; ++pass) {
                blas_check(rocblas_zgemm(hb, rocblas_operation_conjugate_transpose, rocblas_operation_none, kc, ns,
                                         (int)n, &one, rz(V), (int)n, rz(Vn), (int)n, &zero, rz(d_h), kc),
                           "zgemm (V^H W)");
                blas_check(rocblas_zgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, ns, kc, &mone,
                                         rz(V), (int)n, rz(d_h), kc, &one, rz(Vn), (int)n),
                           "zgemm (W - V H)");
                hip_check(hipMemcpyAsync(h2.data(), d_h, sizeof(zc) * kc * ns, hipMemcpyDeviceToHost, st), "D2H");
                hip_check(hipStreamSynchronize(st), "stream sync");
                for (size_t e = 0; e < h.size(); ++e) h[e] += h2[e];
            }
            std::vector<zc> Hn;
            const bool ok = cholqr2(hb, Vn, n, ns, d_g, Hn, st);
            for (int j = 0; j < ns; ++j) {
                for (int i = 0; i < kc; ++i) Hb[(size_t)i + (size_t)(k * ns + j) * M0] = h[(size_t)i + (size_t)j * kc];
                for (int i = 0; i < ns; ++i)
                    Hb[(size_t)(kc + i) + (size_t)(k * ns + j) * M0] = ok ? Hn[(size_t)i + (size_t)j * ns] : zc(0.0, 0.0);
            }
            ++k;
            ++steps;
            // least squares on the leading (k + 1) s x k s block
            const int M = (k + 1) * ns, K = k * ns;
            std::vector<zc> Hk((size_t)M * K), rhs((size_t)M * ns, zc(0.0, 0.0));
            for (int j = 0; j < K; ++j)
                for (int i = 0; i < M; ++i) Hk[(size_t)i + (size_t)j * M] = Hb[(size_t)i + (size_t)j * M0];
            for (int j = 0; j < ns; ++j)
                for (int i = 0; i < ns; ++i) rhs[(size_t)i + (size_t)j * M] = S[(size_t)i + (size_t)j * ns];
            std::vector<double> lsr;
            block_ls(Hk, M, K, rhs, ns, Y, lsr);
            bool done = !fixed;
            for (int c = 0; c < ns; ++c) done &= lsr[c] <= opts->tol * bn[c];
            if (done || !ok) break;
        }
        if (k == 0) break;
        // X += P^-1 (V Y)
        const int K = k * ns;
        hip_check(hipMemcpyAsync(d_y, Y.data(), sizeof(zc) * K * ns, hipMemcpyHostToDevice, st), "H2D");
        blas_check(rocblas_zgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)n, ns, K, &one, rz(V),
                                 (int)n, rz(d_y), K, &zero, rz(tmp), (int)n),
                   "zgemm (V Y)");
        precond(tmp, Wt);
        blas_check(rocblas_zaxpy(hb, (int)blk, &one, rz(Wt), 1, rz(xt), 1), "zaxpy");
        // true residual
        matvec_tree(ctx, H, xt, tmp, ns, slots, st, kAllCols);
        hs::launch_residual(bt, tmp, Wt, n, ns, npart, nchunk, st);
        std::vector<double> pp = download(npart, (size_t)nchunk * ns, st);
        bool all = true;
        for (int c = 0; c < ns; ++c) {
            double r = 0.0;
            for (int ch = 0; ch < nchunk; ++ch) r += pp[(size_t)ch * ns + c];
            rel[c] = bn[c] > 0.0 ? std::sqrt(r) / bn[c] : 0.0;
            all &= rel[c] <= opts->tol;
        }
        if (steps >= budget || (!fixed && all)) break;
    }
    hs::launch_permute(xt, static_cast<cd*>(x), H->d_perm, n, ns, false, st);
    hip_check(hipGetLastError(), "block GMRES launches");
    hip_check(hipStreamSynchronize(st), "stream sync");
    if (P) check_sweep_flag(sw, st);
    bool all_conv = true;
    for (int c = 0; c < ns; ++c) {
        stats[c].iters = steps;
        stats[c].relres = rel[c];
        stats[c].converged = rel[c] <= opts->tol ? 1 : 0;
        if (!std::isfinite(rel[c])) fail(HS_ENUMERIC, "NaN or Inf in the residual");
        all_conv &= stats[c].converged != 0;
    }
    return all_conv ? HS_OK : HS_NOT_CONVERGED;
}

// The paper's transformed system (Eq. 25-28): GMRES on
//   x~ + D^-1 alpha^T Z_F alpha x~ = D^-1 alpha^T b,  x = alpha x~,
// with the identity as right preconditioner, so the iteration monitors the
// transformed left-preconditioned residual; the near-field matvec drops out
// (alpha^T Z_N alpha = D). The true residual of x is computed at the end
// with the full operator and reported in stats.
int32_t solve_transformed(hs_context* ctx, const hs_hmatrix* H, const hs_precond* P, const void* b, void* x,
                          int64_t nrhs, const hs_solve_opts* opts, hs_solve_stats* stats) {
    if (!P || P->block_jacobi) fail(HS_EINVAL, "the transformed system needs a Schur preconditioner (its alpha and D)");
    if (opts->use_x0) fail(HS_EINVAL, "use_x0 is supported by HS_SOLVE_GMRES only");
    const int m = opts->restart;
    if (m < 1 || m > hs::kMaxRankCap) fail(HS_EINVAL, "restart must be in [1, 256]");
    if (!(opts->tol >= 0.0)) fail(HS_EINVAL, "tol must be >= 0");
    const int budget = opts->fixed_iters > 0 ? opts->fixed_iters : (opts->max_iters > 0 ? opts->max_iters : 5000);
    set_device(ctx);
    hipStream_t s = ctx->stream;
    const int64_t n = H->n;
    const int ns = (int)nrhs;
    Owned w;
    w.mem = ctx->mem;
    cd* bt = w.get<cd>(n * ns);
    cd* rhs = w.get<cd>(n * ns);
    cd* xt = w.get<cd>(n * ns);
    cd* u = w.get<cd>(n * ns);
    cd* t2 = w.get<cd>(n * ns);
    cd* slots = w.get<cd>((size_t)H->slot_total * ns);
    // the near slots stay zero: only the far kernels write, so the gather sums Z_F alone
    hip_check(hipMemsetAsync(slots, 0, sizeof(cd) * (size_t)H->near_slot_end * ns, s), "memset");
    GmresWs G;
    G.alloc(w, n, ns, m, false);
    SweepWs sw = make_sweep_ws(w, P, ns, s, ctx);
    std::vector<hs::ColState> hst(ns);
    for (auto& c : hst) {
        std::memset(&c, 0, sizeof(c));
        c.tol = opts->tol;
        c.budget = budget;
        c.fixed = opts->fixed_iters > 0 ? 1 : 0;
    }
    hip_check(hipMemcpyAsync(G.st, hst.data(), sizeof(hs::ColState) * ns, hipMemcpyHostToDevice, s), "H2D");
    hip_check(hipMemsetAsync(xt, 0, sizeof(cd) * n * ns, s), "memset");
    hs::launch_permute(static_cast<const cd*>(b), bt, H->d_perm, n, ns, true, s);
    auto far_only = [&](const cd* in, cd* out, const hs::ColMask& mk) {
        timed(ctx, HS_KT_FAR_MV, s, [&] {
            hs::launch_far_mv(mk, H->d_mv_geom, H->d_mv_rank, H->d_mv_ptr, H->d_mv_slot, H->n_far_wg,
                              (int64_t)H->far_geom.size(), in, n, ns, slots, s);
        });
        hs::launch_gather(mk, H->d_leaf_off, H->d_gptr, H->d_gent, H->nb, slots, n, ns, out, s);
    };
    // right-hand side D^-1 alpha^T b
    alpha_t_tree(ctx, P, bt, t2, ns, sw, s, kAllCols);
    hs::launch_block_dinv(P->sp, t2, nullptr, rhs, ns, s);
    cd* zf = w.get<cd>(n * ns);
    // in -> out = in + D^-1 alpha^T Z_F alpha in (out may not alias in)
    ApplyFn op = [&](const cd* in, cd* out, const hs::ColMask& mk) {
        alpha_tree(ctx, P, in, u, ns, sw, s, mk);
        far_only(u, zf, mk);
        alpha_t_tree(ctx, P, zf, t2, ns, sw, s, mk);
        hs::launch_block_dinv(P->sp, t2, in, out, ns, s);
    };
    ApplyFn ident = [&](const cd* in, cd* out, const hs::ColMask& mk) {
        (void)mk;
        if (in != out) hip_check(hipMemcpyAsync(out, in, sizeof(cd) * n * ns, hipMemcpyDeviceToDevice, s), "D2D");
    };
    gmres_run(G, s, rhs, xt, op, ident, false, false, 4, sw.w.err);
    hst = poll_states(G, sw.w.err, s);
    // x = alpha x~, its true residual with the full operator
    alpha_tree(ctx, P, xt, u, ns, sw, s, kAllCols);
    matvec_tree(ctx, H, u, t2, ns, slots, s, kAllCols);
    hs::launch_residual(bt, t2, G.r, n, ns, G.npart, G.nchunk, s);
    std::vector<double> rp = download(G.npart, (size_t)G.nchunk * ns, s);
    hs::launch_col_norms(bt, n, ns, G.npart, G.nchunk, s);
    std::vector<double> bp = download(G.npart, (size_t)G.nchunk * ns, s);
    hs::launch_permute(u, static_cast<cd*>(x), H->d_perm, n, ns, false, s);
    hip_check(hipGetLastError(), "transformed solve launches");
    check_sweep_flag(sw, s);
    bool all_conv = true;
    for (int c = 0; c < ns; ++c) {
        double rr = 0, bb = 0;
        for (int ch = 0; ch < G.nchunk; ++ch) {
            rr += rp[(size_t)ch * ns + c];
            bb += bp[(size_t)ch * ns + c];
        }
        stats[c].iters = hst[c].total;
        stats[c].relres = bb > 0 ? std::sqrt(rr / bb) : 0.0;
        stats[c].converged = stats[c].relres <= opts->tol ? 1 : 0;
        if (!std::isfinite(stats[c].relres)) fail(HS_ENUMERIC, "NaN or Inf in the residual");
        all_conv &= stats[c].converged != 0;
    }
    return all_conv ? HS_OK : HS_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int32_t hs_solve(hs_context* ctx, const hs_hmatrix* H, const hs_precond* P, const void* b, void* x, int64_t nrhs,
                 const hs_solve_opts* opts, hs_solve_stats* stats) {
    try {
        if (!ctx || !H || !b || !x || !opts || !stats) fail(HS_EINVAL, "NULL argument");
        if (nrhs < 1) fail(HS_EINVAL, "nrhs must be >= 1");
        if (P && P->H != H) fail(HS_EINVAL, "the preconditioner belongs to another H-matrix");
        H->join_far();
        const bool refined = opts->method == HS_SOLVE_GMRES_MIXED_IR;
        const bool mixed = opts->method == HS_SOLVE_FGMRES_MIXED || refined;
        if (opts->method == HS_SOLVE_TRANSFORMED) return solve_transformed(ctx, H, P, b, x, nrhs, opts, stats);
        if (opts->method == HS_SOLVE_BLOCK_GMRES) return solve_block(ctx, H, P, b, x, nrhs, opts, stats);
        if (opts->method != HS_SOLVE_GMRES && !mixed) fail(HS_EINVAL, "unsupported method");
        if (opts->use_x0) {
            if (mixed) fail(HS_EINVAL, "use_x0 is supported by HS_SOLVE_GMRES only");
            hs_solve_item it{H, P, b, x, nrhs};
            return hs_solve_many(ctx, 1, &it, opts, stats);
        }
        if (mixed && !H->c64) fail(HS_EINVAL, "the mixed solve needs an H-matrix built with store_c64");
        if (mixed && P && !P->c64) fail(HS_EINVAL, "the mixed solve needs a preconditioner set up with HS_PREC_MIXED");
        const int m = opts->restart;
        if (m < 1 || m > hs::kMaxRankCap) fail(HS_EINVAL, "restart must be in [1, 256]");
        if (!(opts->tol >= 0.0)) fail(HS_EINVAL, "tol must be >= 0");
        const int m_in = opts->inner_steps > 0 ? opts->inner_steps : 20;
        const double tol_in = opts->inner_tol > 0.0 ? opts->inner_tol : 1e-2;
        if (mixed && m_in > hs::kMaxRankCap) fail(HS_EINVAL, "inner_steps must be in [1, 256]");
        const int budget = opts->fixed_iters > 0 ? opts->fixed_iters : (opts->max_iters > 0 ? opts->max_iters : 5000);
        set_device(ctx);
        hipStream_t s = ctx->stream;
        const int64_t n = H->n;
        const int ns = (int)nrhs;
        Owned w;
        w.mem = ctx->mem;
        cd* bt = w.get<cd>(n * ns);
        cd* xt = w.get<cd>(n * ns);
        cd* slots = w.get<cd>((size_t)H->slot_total * ns);
        GmresWs G;
        G.alloc(w, n, ns, m, mixed && !refined);
        SweepWs sw;
        if (P) sw = make_sweep_ws(w, P, ns, s, ctx);
        std::vector<hs::ColState> hst(ns);
        for (auto& c : hst) {
            std::memset(&c, 0, sizeof(c));
            c.tol = opts->tol;
            c.budget = budget;
            c.fixed = opts->fixed_iters > 0 ? 1 : 0;
        }
        hip_check(hipMemcpyAsync(G.st, hst.data(), sizeof(hs::ColState) * ns, hipMemcpyHostToDevice, s), "H2D");
        hip_check(hipMemsetAsync(xt, 0, sizeof(cd) * n * ns, s), "memset");
        hs::launch_permute(static_cast<const cd*>(b), bt, H->d_perm, n, ns, true, s);
        ApplyFn matvec = [&](const cd* in, cd* out, const hs::ColMask& mk) {
            matvec_tree(ctx, H, in, out, ns, slots, s, mk);
        };
        ApplyFn precond = [&](const cd* in, cd* out, const hs::ColMask& mk) {
            if (P) apply_tree(ctx, P, in, out, ns, sw, s, mk);
            else hip_check(hipMemcpyAsync(out, in, sizeof(cd) * n * ns, hipMemcpyDeviceToDevice, s), "D2D");
        };
        if (!mixed) {
            gmres_run(G, s, bt, xt, matvec, precond, false, false, 4, P ? sw.w.err : nullptr);
        } else {
            ApplyFn matvec32 = [&](const cd* in, cd* out, const hs::ColMask& mk) {
                AuxStream& ax = ctx->aux;
                ax.ensure();
                hip_check(hipEventRecord(ax.fork, s), "hipEventRecord");
                hip_check(hipStreamWaitEvent(ax.s, ax.fork, 0), "hipStreamWaitEvent");
                hs::launch_near_mv(mk, H->d_near_tasks, H->d_near_slot, (int64_t)H->near_tasks.size(), H->d_near32,
                                   in, n, ns, slots, ax.s);
                hs::launch_far_mv(mk, H->d_mv_geom, H->d_mv_rank, H->d_mv_ptr32, H->d_mv_slot, H->n_far_wg,
                                  (int64_t)H->far_geom.size(), in, n, ns, slots, s);
                hip_check(hipEventRecord(ax.join, ax.s), "hipEventRecord");
                hip_check(hipStreamWaitEvent(s, ax.join, 0), "hipStreamWaitEvent");
                hs::launch_gather(mk, H->d_leaf_off, H->d_gptr, H->d_gent, H->nb, slots, n, ns, out, s);
            };
            ApplyFn precond32 = [&](const cd* in, cd* out, const hs::ColMask& mk) {
                if (!P) {
                    hip_check(hipMemcpyAsync(out, in, sizeof(cd) * n * ns, hipMemcpyDeviceToDevice, s), "D2D");
                    return;
                }
                sw.epoch_f += 1;
                sw.epoch_b += 1;
                sweeps_begin(ctx->device, s);
                hs::launch_sweep(true, mk, P->sp32, P->items, in, out, ns, sw.w, sw.epoch_f, s);
                hs::launch_sweep(false, mk, P->sp32, P->items, in, out, ns, sw.w, sw.epoch_b, s);
                sweeps_end(ctx->device, s);
            };
            if (refined) {
                // Arnoldi on the complex64 copies (FP32 arithmetic, FP64
                // vectors and Givens), the true residual on the FP64 operator
                gmres_run(G, s, bt, xt, matvec32, precond32, false, false, 4, P ? sw.w.err : nullptr, &matvec);
            } else {
                // inner solves: complex64 operator and preconditioner copies, FP64 vectors
                GmresWs Gi;
                Gi.alloc(w, n, ns, m_in, false);
                // one flexible preconditioning step: z = approximate Z^-1 v for the
                // columns still stepping in the outer cycle
                ApplyFn inner = [&](const cd* in, cd* out, const hs::ColMask& mk) {
                    hip_check(hipMemsetAsync(out, 0, sizeof(cd) * n * ns, s), "memset");
                    hs::launch_col_init(Gi.st, mk.st, ns, tol_in, m_in, s);
                    gmres_run(Gi, s, in, out, matvec32, precond32, false, true, 4, P ? sw.w.err : nullptr);
                };
                gmres_run(G, s, bt, xt, matvec, inner, true, false, 4, P ? sw.w.err : nullptr);
            }
        }
        hst = poll_states(G, P ? sw.w.err : nullptr, s);
        hs::launch_permute(xt, static_cast<cd*>(x), H->d_perm, n, ns, false, s);
        hip_check(hipGetLastError(), "permute launch");
        hip_check(hipStreamSynchronize(s), "stream sync");
        bool all_conv = true;
        for (int c = 0; c < ns; ++c) {
            stats[c].iters = hst[c].total;
            stats[c].relres = hst[c].relres;
            stats[c].converged = hst[c].relres <= opts->tol ? 1 : 0;
            if (!std::isfinite(hst[c].relres)) fail(HS_ENUMERIC, "NaN or Inf in the residual");
            all_conv &= stats[c].converged != 0;
        }
        return all_conv ? HS_OK : HS_NOT_CONVERGED;
    } catch (const Error& e) {
        return set_error(e);
    }
}

// ---- multi-geometry solves: lanes in lockstep -------------------------------------------

}  // extern "C"

namespace {

// The solve state of one geometry inside a multi-geometry solve: ns column
// slots of a right-preconditioned GMRES(m) on tree-order vectors, on one
// stream. A slot holds one right-hand side from its start (x = 0, or the
// caller's x0) until its column is done; in serving, a freed slot takes the
// next pending column at a cycle boundary. Columns are independent Krylov
// spaces: a column's arithmetic does not depend on the other slots.
struct Lane {
    const hs_hmatrix* H = nullptr;
    const hs_precond* P = nullptr;
    hipStream_t s = nullptr;
    bool aux = false;          // near matvec on the context's auxiliary stream
    int ns = 0, m = 0;
    Owned w;
    cd *bt = nullptr, *xt = nullptr, *slots = nullptr;
    int* d_cols = nullptr;     // slot list for the column starts
    GmresWs G;
    SweepWs sw;
    std::vector<hs::ColState> st;   // host copy at the last poll
    bool ran = false;          // took part in the current cycle
    bool stepping = false;     // some column still stepping in the current cycle
    int err = 0;
};

// Device bytes a lane allocates (the same sizes as lane_alloc, each rounded
// up to the allocator's 256-byte granule).
int64_t lane_bytes(const hs_hmatrix* H, const hs_precond* P, int ns, int m) {
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    const int64_t n = H->n, nn = n * ns, c = 16;
    const int64_t nch = hs::gmres_nchunk(n);
    int64_t b = up(nn * c) * 2 + up(H->slot_total * ns * c) + up(ns * 4);
    b += up(nn * c) * 3 + up((m + 1) * nn * c) + up((int64_t)(m + 1) * m * ns * c) + up(m * ns * 8) + up(m * ns * c) +
         up((m + 1) * ns * c) + up(m * ns * c) + up(nch * (m + 1) * ns * c) + up(nch * ns * 8) + up(ns * 8) +
         up(ns * (int64_t)sizeof(hs::ColState));
    if (P) {
        b += up(4) + up(nn * c) * 4 + up(std::max<int64_t>(P->fslot_total, 1) * ns * c) +
             up(std::max<int64_t>(P->bslot_total, 1) * ns * c) +
             up(((int64_t)4 * hs::kCntPad * P->nchunk + 2 * P->nb) * 4) + up(16) + up(4 * nn * 8) * 2;
    }
    return b;
}

void lane_alloc(hs_context* ctx, Lane& L, const hs_hmatrix* H, const hs_precond* P, int ns, int m, hipStream_t s,
                bool aux) {
    H->join_far();
    L.H = H;
    L.P = P;
    L.s = s;
    L.aux = aux;
    L.ns = ns;
    L.m = m;
    L.w.mem = ctx->mem;
    const int64_t n = H->n;
    L.bt = L.w.get<cd>(n * ns);
    L.xt = L.w.get<cd>(n * ns);
    L.slots = L.w.get<cd>((size_t)H->slot_total * ns);
    L.d_cols = L.w.get<int>(ns);
    L.G.alloc(L.w, n, ns, m, false);
    if (P) L.sw = make_sweep_ws(L.w, P, ns, s, ctx);
    // every slot starts free (done)
    L.st.assign(ns, hs::ColState{});
    for (auto& c : L.st) c.done = 1;
    hip_check(hipMemcpyAsync(L.G.st, L.st.data(), sizeof(hs::ColState) * ns, hipMemcpyHostToDevice, s), "H2D");
}

void lane_matvec(hs_context* ctx, Lane& L, const cd* in, cd* out, const hs::ColMask& mk) {
    if (L.aux) {
        matvec_tree(ctx, L.H, in, out, L.ns, L.slots, L.s, mk);
        return;
    }
    // near and far one after the other on the lane's stream (disjoint slots)
    const hs_hmatrix* H = L.H;
    timed(ctx, HS_KT_NEAR_MV, L.s, [&] {
        hs::launch_near_mv(mk, H->d_near_tasks, H->d_near_slot, (int64_t)H->near_tasks.size(), H->d_near, in, H->n,
                           L.ns, L.slots, L.s);
    });
    timed(ctx, HS_KT_FAR_MV, L.s, [&] {
        hs::launch_far_mv(mk, H->d_mv_geom, H->d_mv_rank, H->d_mv_ptr, H->d_mv_slot, H->n_far_wg,
                          (int64_t)H->far_geom.size(), in, H->n, L.ns, L.slots, L.s);
    });
    hs::launch_gather(mk, H->d_leaf_off, H->d_gptr, H->d_gent, H->nb, L.slots, H->n, L.ns, out, L.s);
}

void lane_precond(hs_context* ctx, Lane& L, const cd* in, cd* out, const hs::ColMask& mk) {
    if (L.P) apply_tree(ctx, L.P, in, out, L.ns, L.sw, L.s, mk);
    else hip_check(hipMemcpyAsync(out, in, sizeof(cd) * L.H->n * L.ns, hipMemcpyDeviceToDevice, L.s), "D2D");
}

// Start the listed slots (their b already in bt, tree order) from x = 0:
// r = b - Z 0 = b for them (every other column's r is recomputed from the
// Z x of the last cycle end, unchanged), then their fresh states. The
// partials are those of ||b||^2, as a solve's first cycle start uses.
void lane_start_cols(Lane& L, const std::vector<int>& cols, const hs_solve_opts& o, int budget) {
    if (cols.empty()) return;
    const int64_t n = L.H->n;
    for (int c : cols) {
        hip_check(hipMemsetAsync(L.xt + (int64_t)c * n, 0, sizeof(cd) * n, L.s), "memset");
        hip_check(hipMemsetAsync(L.G.tmp + (int64_t)c * n, 0, sizeof(cd) * n, L.s), "memset");
    }
    hip_check(hipMemcpyAsync(L.d_cols, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice, L.s), "H2D");
    hs::launch_residual(L.bt, L.G.tmp, L.G.r, n, L.ns, L.G.npart, L.G.nchunk, L.s);
    hs::launch_col_start(L.G.npart, L.G.nchunk, L.G.st, L.ns, L.d_cols, (int)cols.size(), o.tol, budget,
                         o.fixed_iters > 0 ? 1 : 0, L.s);
    // the slots are live from now on (the host copy catches up at the next poll)
    for (int c : cols) L.st[c].done = 0;
}

// Start every slot from the caller's x0 (already in xt): ||b|| from b, then
// r = b - Z x0.
void lane_start_x0(hs_context* ctx, Lane& L, const hs_solve_opts& o, int budget) {
    const int64_t n = L.H->n;
    std::vector<int> cols(L.ns);
    for (int c = 0; c < L.ns; ++c) cols[c] = c;
    hip_check(hipMemcpyAsync(L.d_cols, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice, L.s), "H2D");
    hs::launch_col_norms(L.bt, n, L.ns, L.G.npart, L.G.nchunk, L.s);
    hs::launch_col_start(L.G.npart, L.G.nchunk, L.G.st, L.ns, L.d_cols, L.ns, o.tol, budget, o.fixed_iters > 0 ? 1 : 0,
                         L.s);
    lane_matvec(ctx, L, L.xt, L.G.tmp, kAllCols);
    hs::launch_residual(L.bt, L.G.tmp, L.G.r, n, L.ns, L.G.npart, L.G.nchunk, L.s);
    for (auto& c : L.st) c.done = 0;
}

bool lane_live(const Lane& L) {
    for (const auto& c : L.st)
        if (!c.done) return true;
    return false;
}

// Column states of the given lanes to the host (one synchronisation per
// stream), with the sweeps' error flags.
void lanes_poll(std::vector<Lane*>& ls) {
    for (Lane* L : ls) {
        hip_check(hipMemcpyAsync(L->st.data(), L->G.st, sizeof(hs::ColState) * L->ns, hipMemcpyDeviceToHost, L->s),
                  "D2H");
        L->err = 0;
        if (L->P) hip_check(hipMemcpyAsync(&L->err, L->sw.w.err, sizeof(int), hipMemcpyDeviceToHost, L->s), "D2H");
    }
    for (Lane* L : ls) hip_check(hipStreamSynchronize(L->s), "stream sync");
    for (Lane* L : ls)
        if (L->err)
            fail(HS_ETIMEOUT, "a device-side wait of the preconditioner sweeps exceeded the context's wait limit");
}

// One restart cycle of every lane with a live column, in lockstep: the
// lanes' launches alternate step by step, each lane on its own stream, and a
// poll reads all of them at once. Same arithmetic per lane as gmres_run.
void lanes_cycle(hs_context* ctx, std::vector<Lane*>& lanes, int poll) {
    std::vector<Lane*> run;
    for (Lane* L : lanes) {
        L->ran = lane_live(*L);
        L->stepping = L->ran;
        if (!L->ran) continue;
        run.push_back(L);
        if (!L->G.ring || L->G.ring->ns != L->ns) L->G.ring = std::make_shared<PollRing>(L->ns);
        L->G.ring->reset();
        hip_check(hipMemsetAsync(L->G.Hh, 0, sizeof(cd) * L->G.ldh * L->ns, L->s), "memset");
        hs::launch_cycle_start(L->G.r, L->G.V, L->H->n, L->G.g, L->m, L->G.npart, L->G.nchunk, L->G.st, L->H->n, L->ns,
                               false, L->s);
    }
    if (run.empty()) return;
    int m = 0;
    for (Lane* L : run) m = std::max(m, L->m);
    for (int j = 0; j < m; ++j) {
        for (Lane* L : run) {
            if (!L->stepping || j >= L->m) continue;
            GmresWs& G = L->G;
            const int64_t n = G.n, vs = G.vstride;
            const hs::ColMask active{G.st, 1, 0};
            lane_precond(ctx, *L, G.V + j * vs, G.tmp, active);
            lane_matvec(ctx, *L, G.tmp, G.wv, active);
            hs::launch_dots(G.V, n, vs, j + 1, G.wv, n, G.ns, G.st, G.partial, G.nchunk, L->s);
            hs::launch_basis_update(G.V, n, vs, j + 1, G.partial, G.nchunk, G.wv, n, G.ns, G.st, G.Hh, G.ldh, G.m + 1,
                                    j, false, nullptr, L->s);
            hs::launch_dots(G.V, n, vs, j + 1, G.wv, n, G.ns, G.st, G.partial, G.nchunk, L->s);
            hs::launch_basis_update(G.V, n, vs, j + 1, G.partial, G.nchunk, G.wv, n, G.ns, G.st, G.Hh, G.ldh, G.m + 1,
                                    j, true, G.npart, L->s);
            hs::launch_givens_scale(G.Hh, G.ldh, G.m, j, G.csv, G.snv, G.g, G.npart, G.nchunk, G.st, G.ns, G.wv,
                                    G.V + (j + 1) * vs, n, n, L->s);
        }
        if ((j + 1) % poll == 0 && j + 1 < m) {
            std::vector<Lane*> live;
            for (Lane* L : run)
                if (L->stepping && j + 1 < L->m) live.push_back(L);
            if (live.empty()) break;
            for (Lane* L : live) hip_check(hipGetLastError(), "inner launches");
            // one poll behind, as in gmres_run: a lane stops stepping once
            // its previous poll point saw no column still stepping
            bool any = false;
            for (Lane* L : live) {
                L->stepping = !L->G.ring->poll(L->G.st, L->P ? L->sw.w.err : nullptr, L->s);
                any |= L->stepping;
            }
            if (!any) break;
        }
    }
    for (Lane* L : run) {
        GmresWs& G = L->G;
        const int64_t n = G.n, vs = G.vstride;
        const hs::ColMask stepped{G.st, 2, 0};
        hs::launch_lsq(G.Hh, G.ldh, G.m, G.g, G.y, G.st, G.ns, L->s);
        hs::launch_combine(G.V, n, vs, G.y, G.m, G.tmp, n, G.ns, G.st, L->s);
        lane_precond(ctx, *L, G.tmp, G.wv, stepped);
        hs::launch_axpy_x(L->xt, G.wv, n, G.ns, G.st, L->s);
        lane_matvec(ctx, *L, L->xt, G.tmp, stepped);
        hs::launch_residual(L->bt, G.tmp, G.r, n, G.ns, G.npart, G.nchunk, L->s);
        hs::launch_cycle_end(G.npart, G.nchunk, G.st, G.ns, L->s);
        hip_check(hipGetLastError(), "cycle launches");
    }
    lanes_poll(run);
}

// Streams for lanes: lane 0 on the context's stream, the others spread over
// up to three library-owned streams (default priority) that first wait for
// everything already queued on the context's stream.
struct LaneStreams {
    hipStream_t s[3] = {};
    hipEvent_t ev[4] = {};
    int used = 0;
    int device = -1;
    void ensure(int k) {
        if (device < 0) hip_check(hipGetDevice(&device), "hipGetDevice");
        for (int i = used; i < k; ++i) {
            hip_check(hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking), "hipStreamCreateWithFlags");
            hip_check(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming), "hipEventCreateWithFlags");
        }
        if (!ev[3]) hip_check(hipEventCreateWithFlags(&ev[3], hipEventDisableTiming), "hipEventCreateWithFlags");
        used = std::max(used, k);
    }
    ~LaneStreams() {
        // the sweeps' cross-stream order must not keep a stream about to go
        if (device >= 0)
            for (auto x : s)
                if (x) sweeps_release(device, x);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto x : s)
            if (x) (void)hipStreamDestroy(x);
    }
};

hipStream_t lane_stream(hs_context* ctx, LaneStreams& ls, size_t i) {
    if (i == 0) return ctx->stream;
    return ls.s[(i - 1) % 3];
}

// Extra streams wait for the context's stream (inputs ready).
void lanes_fork(hs_context* ctx, LaneStreams& ls, size_t nlanes) {
    const int k = (int)std::min<size_t>(nlanes > 0 ? nlanes - 1 : 0, 3);
    if (k == 0) return;
    ls.ensure(k);
    hip_check(hipEventRecord(ls.ev[3], ctx->stream), "hipEventRecord");
    for (int i = 0; i < k; ++i) hip_check(hipStreamWaitEvent(ls.s[i], ls.ev[3], 0), "hipStreamWaitEvent");
}

// The context's stream waits for the extra streams (outputs ready).
void lanes_join(hs_context* ctx, LaneStreams& ls) {
    for (int i = 0; i < ls.used; ++i) {
        hip_check(hipEventRecord(ls.ev[i], ls.s[i]), "hipEventRecord");
        hip_check(hipStreamWaitEvent(ctx->stream, ls.ev[i], 0), "hipStreamWaitEvent");
    }
}

void check_solve_opts(const hs_solve_opts* o) {
    if (o->method != HS_SOLVE_GMRES) fail(HS_EINVAL, "only HS_SOLVE_GMRES runs on the multi-geometry engine");
    if (o->restart < 1 || o->restart > hs::kMaxRankCap) fail(HS_EINVAL, "restart must be in [1, 256]");
    if (!(o->tol >= 0.0)) fail(HS_EINVAL, "tol must be >= 0");
}

int solve_budget(const hs_solve_opts* o) {
    return o->fixed_iters > 0 ? o->fixed_iters : (o->max_iters > 0 ? o->max_iters : 5000);
}

}  // namespace

extern "C" {

int32_t hs_solve_many(hs_context* ctx, int64_t nitems, const hs_solve_item* items, const hs_solve_opts* opts,
                      hs_solve_stats* stats) {
    try {
        if (!ctx || !items || !opts || !stats) fail(HS_EINVAL, "NULL argument");
        if (nitems < 1) fail(HS_EINVAL, "nitems must be >= 1");
        check_solve_opts(opts);
        for (int64_t i = 0; i < nitems; ++i) {
            const hs_solve_item& it = items[i];
            if (!it.H || !it.b || !it.x) fail(HS_EINVAL, "item " + std::to_string(i) + ": NULL H, b or x");
            it.H->join_far();
            if (it.nrhs < 1 || it.nrhs > (1 << 20)) fail(HS_EINVAL, "item " + std::to_string(i) + ": bad nrhs");
            if (it.P && it.P->H != it.H) fail(HS_EINVAL, "item " + std::to_string(i) + ": P belongs to another H");
        }
        set_device(ctx);
        const int budget = solve_budget(opts);
        LaneStreams ls;
        std::vector<std::unique_ptr<Lane>> lanes;
        lanes_fork(ctx, ls, (size_t)nitems);
        for (int64_t i = 0; i < nitems; ++i) {
            const hs_solve_item& it = items[i];
            auto L = std::make_unique<Lane>();
            lane_alloc(ctx, *L, it.H, it.P, (int)it.nrhs, opts->restart, lane_stream(ctx, ls, (size_t)i), i == 0);
            hs::launch_permute(static_cast<const cd*>(it.b), L->bt, it.H->d_perm, it.H->n, it.nrhs, true, L->s);
            if (opts->use_x0) {
                hs::launch_permute(static_cast<const cd*>(it.x), L->xt, it.H->d_perm, it.H->n, it.nrhs, true, L->s);
                lane_start_x0(ctx, *L, *opts, budget);
            } else {
                std::vector<int> cols((size_t)it.nrhs);
                for (int c = 0; c < (int)it.nrhs; ++c) cols[c] = c;
                lane_start_cols(*L, cols, *opts, budget);
            }
            lanes.push_back(std::move(L));
        }
        std::vector<Lane*> lp;
        for (auto& L : lanes) lp.push_back(L.get());
        for (;;) {
            bool any = false;
            for (Lane* L : lp) any |= lane_live(*L);
            if (!any) break;
            lanes_cycle(ctx, lp, 4);
        }
        int64_t k = 0;
        bool all_conv = true;
        for (int64_t i = 0; i < nitems; ++i) {
            Lane& L = *lanes[i];
            hs::launch_permute(L.xt, static_cast<cd*>(items[i].x), L.H->d_perm, L.H->n, L.ns, false, L.s);
            for (int c = 0; c < L.ns; ++c, ++k) {
                stats[k].iters = L.st[c].total;
                stats[k].relres = L.st[c].relres;
                stats[k].converged = L.st[c].relres <= opts->tol ? 1 : 0;
                if (!std::isfinite(L.st[c].relres)) fail(HS_ENUMERIC, "NaN or Inf in the residual");
                all_conv &= stats[k].converged != 0;
            }
        }
        for (auto& L : lanes) hip_check(hipGetLastError(), "permute launch");
        lanes_join(ctx, ls);
        for (auto& L : lanes) hip_check(hipStreamSynchronize(L->s), "stream sync");
        return all_conv ? HS_OK : HS_NOT_CONVERGED;
    } catch (const Error& e) {
        (void)hipDeviceSynchronize();
        return set_error(e);
    }
}

// ---- serving: continuous batching ----------------------------------------------------------

}  // extern "C"

struct hs_server {
    hs_context* ctx = nullptr;
    int64_t budget = 0, used = 0;
    int32_t slots = 32;           // column slots per geometry
    hs_solve_opts opts{};
    LaneStreams ls;
    struct Geometry {
        const hs_hmatrix* H = nullptr;
        const hs_precond* P = nullptr;
        hs_hmatrix* Hown = nullptr;   // built by the server (hs_server_add_geometry)
        hs_precond* Pown = nullptr;
        std::unique_ptr<Lane> lane;   // allocated at the geometry's first request
        std::vector<std::pair<int64_t, int32_t>> slot_req;   // (request, column) per slot, request -1 = free
        int64_t bytes = 0;
    };
    std::vector<Geometry> geos;
    std::vector<const hs_hmatrix*> counted_h;
    struct Request {
        int32_t geometry = 0, ncols = 0, admitted = 0, retired = 0;
        const cd* b = nullptr;
        cd* x = nullptr;
        hs_request_stats st{};
    };
    std::vector<Request> reqs;
    std::vector<int64_t> pending;   // not yet (fully) admitted, submission order
    ~hs_server() {
        if (ctx) (void)hipSetDevice(ctx->device);
        for (auto& g : geos) {
            g.lane.reset();
            if (g.Pown) hs_precond_destroy(g.Pown);
            if (g.Hown) hs_hmatrix_destroy(g.Hown);
        }
    }
};

namespace {
double server_clock() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int32_t server_take(hs_server* s, const hs_hmatrix* H, const hs_precond* P, hs_hmatrix* Hown, hs_precond* Pown,
                    int64_t add, int32_t* geometry) {
    s->used += add;
    if (std::find(s->counted_h.begin(), s->counted_h.end(), H) == s->counted_h.end()) s->counted_h.push_back(H);
    hs_server::Geometry g;
    g.H = H;
    g.P = P;
    g.Hown = Hown;
    g.Pown = Pown;
    g.bytes = add;
    g.slot_req.assign(s->slots, {-1, 0});
    s->geos.push_back(std::move(g));
    *geometry = (int32_t)s->geos.size() - 1;
    return HS_OK;
}
}  // namespace

extern "C" {

double hs_server_clock(void) { return server_clock(); }

int32_t hs_server_create(hs_context* ctx, int64_t device_budget_bytes, int32_t slots_per_geometry,
                         const hs_solve_opts* opts, hs_server** out) {
    try {
        if (!ctx || !opts || !out) fail(HS_EINVAL, "NULL argument");
        *out = nullptr;
        if (device_budget_bytes <= 0) fail(HS_EINVAL, "device budget must be positive");
        if (slots_per_geometry < 1 || slots_per_geometry > 1024) fail(HS_EINVAL, "slots_per_geometry must be in [1, 1024]");
        check_solve_opts(opts);
        if (opts->use_x0) fail(HS_EINVAL, "served columns start from x = 0");
        auto* s = new hs_server;
        s->ctx = ctx;
        s->budget = device_budget_bytes;
        s->slots = slots_per_geometry;
        s->opts = *opts;
        *out = s;
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_server_admit(hs_server* s, const hs_hmatrix* H, const hs_precond* P, int32_t* geometry) {
    try {
        if (!s || !H || !geometry) fail(HS_EINVAL, "NULL argument");
        if (P && P->H != H) fail(HS_EINVAL, "the preconditioner belongs to another H-matrix");
        H->join_far();
        int64_t add = (P ? P->own.bytes : 0) + lane_bytes(H, P, s->slots, s->opts.restart);
        const bool h_new = std::find(s->counted_h.begin(), s->counted_h.end(), H) == s->counted_h.end();
        if (h_new) add += H->own.bytes;
        if (s->used + add > s->budget)
            fail(HS_ENOMEM, "admission refused: the geometry's device footprint (" + std::to_string(add) +
                                " bytes with its solve workspace) exceeds the remaining budget");
        return server_take(s, H, P, nullptr, nullptr, add, geometry);
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_server_add_geometry(hs_server* s, const double* points_host, int64_t n, double k, double self_h,
                               const hs_build_opts* bopts, const hs_precond_opts* popts, int64_t* estimate,
                               int32_t* geometry) {
    hs_hmatrix* H = nullptr;
    hs_precond* P = nullptr;
    try {
        if (!s || !points_host || !bopts || !geometry) fail(HS_EINVAL, "NULL argument");
        if (n < 1) fail(HS_EINVAL, "n must be >= 1");
        // 1. footprint from the host plan, before any device allocation
        hs_plan* plan = nullptr;
        int32_t rc = hs_plan_create(points_host, n, bopts->leaf_max, popts ? popts->ordering : HS_ORDER_RCM, &plan);
        if (rc != HS_OK) return rc;
        std::unique_ptr<hs_plan, void (*)(hs_plan*)> pg(plan, hs_plan_destroy);
        hs_info inf;
        hs_plan_query(plan, &inf);
        const int64_t est = inf.bytes_estimate;
        if (estimate) *estimate = est;
        if (s->used + est > s->budget)
            fail(HS_ENOMEM, "admission refused before allocation: the plan's footprint estimate (" +
                                std::to_string(est) + " bytes) exceeds the remaining budget");
        // 2. build on the device, then charge the actual footprint
        set_device(s->ctx);
        Owned tmp;
        tmp.mem = s->ctx->mem;
        double* d_pts = tmp.get<double>((size_t)n * 3);
        hip_check(hipMemcpyAsync(d_pts, points_host, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s->ctx->stream),
                  "H2D");
        rc = hs_h_build(s->ctx, d_pts, n, k, self_h, bopts, &H);
        if (rc != HS_OK) return rc;
        if (popts) {
            rc = hs_precond_setup(s->ctx, H, popts, &P);
            if (rc != HS_OK) {
                hs_hmatrix_destroy(H);
                return rc;
            }
        }
        tmp.release();
        H->join_far();
        const int64_t add = H->own.bytes + (P ? P->own.bytes : 0) + lane_bytes(H, P, s->slots, s->opts.restart);
        if (s->used + add > s->budget)
            fail(HS_ENOMEM, "admission refused: the built geometry needs " + std::to_string(add) +
                                " bytes, more than the remaining budget (the plan estimated " + std::to_string(est) +
                                ")");
        rc = server_take(s, H, P, H, P, add, geometry);
        H = nullptr;
        P = nullptr;
        return rc;
    } catch (const Error& e) {
        if (P) hs_precond_destroy(P);
        if (H) hs_hmatrix_destroy(H);
        return set_error(e);
    }
}

int32_t hs_server_submit(hs_server* s, int32_t geometry, const void* b, void* x, int32_t ncols, double t_arrival,
                         int64_t* request) {
    try {
        if (!s || !b || !x || !request) fail(HS_EINVAL, "NULL argument");
        if (geometry < 0 || geometry >= (int32_t)s->geos.size()) fail(HS_EINVAL, "unknown geometry");
        if (ncols < 1 || ncols > s->slots) fail(HS_EINVAL, "ncols must be in [1, slots_per_geometry]");
        hs_server::Request r;
        r.geometry = geometry;
        r.ncols = ncols;
        r.b = static_cast<const cd*>(b);
        r.x = static_cast<cd*>(x);
        r.st.geometry = geometry;
        r.st.ncols = ncols;
        r.st.t_arrival = t_arrival;
        r.st.converged = 1;
        s->reqs.push_back(r);
        *request = (int64_t)s->reqs.size() - 1;
        s->pending.push_back(*request);
        return HS_OK;
    } catch (const Error& e) {
        return set_error(e);
    }
}

int32_t hs_server_step(hs_server* s, int32_t* columns_served) {
    try {
        if (!s || !columns_served) fail(HS_EINVAL, "NULL argument");
        *columns_served = 0;
        hs_context* ctx = s->ctx;
        set_device(ctx);
        const int budget = solve_budget(&s->opts);
        // 1. admission at the cycle boundary: per geometry, pending requests in
        //    arrival order take free slots while the oldest one fits (no later
        //    request of that geometry jumps ahead of it)
        auto older = [&](int64_t p, int64_t q) {
            const auto &a = s->reqs[p].st, &b = s->reqs[q].st;
            return a.t_arrival != b.t_arrival ? a.t_arrival < b.t_arrival : p < q;
        };
        std::vector<int64_t> order(s->pending);
        std::stable_sort(order.begin(), order.end(), older);
        std::vector<char> blocked(s->geos.size(), 0);
        std::vector<std::vector<int>> fresh(s->geos.size());
        std::vector<std::pair<int64_t, int>> admit;   // (request, geometry) admitted now
        std::vector<int> nfree(s->geos.size(), 0);
        for (size_t gi = 0; gi < s->geos.size(); ++gi)
            for (auto& sr : s->geos[gi].slot_req) nfree[gi] += sr.first < 0 ? 1 : 0;
        for (int64_t q : order) {
            auto& r = s->reqs[q];
            if (blocked[r.geometry]) continue;
            if (nfree[r.geometry] < r.ncols) {
                blocked[r.geometry] = 1;
                continue;
            }
            nfree[r.geometry] -= r.ncols;
            admit.push_back({q, r.geometry});
            r.st.t_start = server_clock();
            auto& g = s->geos[r.geometry];
            if (!g.lane) {
                size_t idx = 0;
                for (auto& gg : s->geos) idx += gg.lane ? 1 : 0;
                if (idx > 0) s->ls.ensure(std::min<int>((int)idx, 3));
                g.lane = std::make_unique<Lane>();
                lane_alloc(ctx, *g.lane, g.H, g.P, s->slots, s->opts.restart, lane_stream(ctx, s->ls, idx), idx == 0);
            }
        }
        // lanes on the library's streams follow the caller's work (the submitted b)
        if (!admit.empty() && s->ls.used > 0) {
            hip_check(hipEventRecord(s->ls.ev[3], ctx->stream), "hipEventRecord");
            for (int i = 0; i < s->ls.used; ++i)
                hip_check(hipStreamWaitEvent(s->ls.s[i], s->ls.ev[3], 0), "hipStreamWaitEvent");
        }
        for (auto& a : admit) {
            auto& r = s->reqs[a.first];
            auto& g = s->geos[a.second];
            Lane& L = *g.lane;
            int c = 0;
            for (int sl = 0; sl < s->slots && c < r.ncols; ++sl) {
                if (g.slot_req[sl].first >= 0) continue;
                g.slot_req[sl] = {a.first, c};
                hs::launch_permute(r.b + (int64_t)c * g.H->n, L.bt + (int64_t)sl * g.H->n, g.H->d_perm, g.H->n, 1, true,
                                   L.s);
                fresh[a.second].push_back(sl);
                ++c;
            }
            r.admitted = r.ncols;
        }
        std::vector<int64_t> rest;
        for (int64_t q : s->pending)
            if (s->reqs[q].admitted < s->reqs[q].ncols) rest.push_back(q);
        s->pending.swap(rest);
        std::vector<Lane*> lanes;
        for (size_t gi = 0; gi < s->geos.size(); ++gi) {
            auto& g = s->geos[gi];
            if (!g.lane) continue;
            lane_start_cols(*g.lane, fresh[gi], s->opts, budget);
            lanes.push_back(g.lane.get());
        }
        // 2. one restart cycle of every geometry with live columns
        lanes_cycle(ctx, lanes, 4);
        // 3. retire finished columns into their requests' x
        std::vector<int64_t> finished;
        int32_t served = 0;
        for (auto& g : s->geos) {
            if (!g.lane) continue;
            Lane& L = *g.lane;
            for (int sl = 0; sl < s->slots; ++sl) {
                auto& sr = g.slot_req[sl];
                if (sr.first < 0 || !L.st[sl].done) continue;
                auto& r = s->reqs[sr.first];
                hs::launch_permute(L.xt + (int64_t)sl * g.H->n, r.x + (int64_t)sr.second * g.H->n, g.H->d_perm, g.H->n,
                                   1, false, L.s);
                const auto& cs = L.st[sl];
                r.st.iters = std::max(r.st.iters, cs.total);
                r.st.relres = std::max(r.st.relres, cs.relres);
                if (!(cs.relres <= s->opts.tol)) r.st.converged = 0;
                if (++r.retired == r.ncols) finished.push_back(sr.first);
                sr = {-1, 0};
                ++served;
            }
        }
        for (auto& g : s->geos)
            if (g.lane) hip_check(hipStreamSynchronize(g.lane->s), "stream sync");
        const double t = server_clock();
        for (int64_t q : finished) {
            s->reqs[q].st.t_done = t;
            s->reqs[q].st.done = 1;
        }
        *columns_served = served;
        return HS_OK;
    } catch (const Error& e) {
        (void)hipDeviceSynchronize();
        return set_error(e);
    }
}

int32_t hs_server_pending(const hs_server* s, int64_t* requests, int64_t* columns) {
    if (!s || !requests || !columns) { g_last_error = "NULL argument"; return HS_EINVAL; }
    // requests not done: queued, or admitted with columns still running
    int64_t r = 0, c = 0;
    for (const auto& q : s->reqs)
        if (!q.st.done) {
            ++r;
            c += q.ncols - q.retired;
        }
    *requests = r;
    *columns = c;
    return HS_OK;
}

int32_t hs_server_request(const hs_server* s, int64_t request, hs_request_stats* out) {
    if (!s || !out) { g_last_error = "NULL argument"; return HS_EINVAL; }
    if (request < 0 || request >= (int64_t)s->reqs.size()) { g_last_error = "unknown request"; return HS_EINVAL; }
    *out = s->reqs[request].st;
    return HS_OK;
}

int32_t hs_server_geometry(const hs_server* s, int32_t geometry, hs_hmatrix const** H, hs_precond const** P,
                           int64_t* bytes) {
    if (!s || geometry < 0 || geometry >= (int32_t)s->geos.size()) { g_last_error = "unknown geometry"; return HS_EINVAL; }
    if (H) *H = s->geos[geometry].H;
    if (P) *P = s->geos[geometry].P;
    if (bytes) *bytes = s->geos[geometry].bytes;
    return HS_OK;
}

void hs_server_destroy(hs_server* s) { delete s; }

}  // extern "C"
