// Preconditioner apply P^-1 v = alpha D^-1 alpha^T v (Eq. 23, 24 and 28):
//
//  forward   y_j = v_j + sum_{k < j, j in S_k} alpha_kj^T y_k   (k ascending)
//            zt_j = D_j^-1 y_j
//  backward  z_k = zt_k + sum_{j in S_k} alpha_kj z_j             (k descending)
//
// Under a bandwidth-reducing order each block row depends on the one before
// it, so both sweeps are chains of nb dependent steps. Consecutive rows are
// grouped into chunks; with Linv_c the explicit inverse of chunk c's unit
// lower-triangular diagonal part and C_c its coupling to a folded range of
// earlier points (all of chunk c-1, then the coupled blocks of earlier chunks,
// nearest first, up to kFoldCols columns),
//   forward   y_c = Linv_c r_c + (Linv_c C_c) y_range
//   backward  z_c = Linv_c^T r'_c + (Linv_c^T C'_c) z_range
// where r, r' gather the terms of the entries outside the range. Phase A of
// a block row gathers those terms (they are ready well before they are
// needed); phase B applies a row's slice of the two dense products, so the
// chain advances one dense row-block product per chunk. The operator is
// unchanged; only the evaluation order of the triangular solves differs.
//
// The terms outside the range are pushed: as soon as a chunk is
// final, a wavefront per far entry (k, j) computes alpha_kj^T y_k (forward)
// or alpha_kj z_j (backward) into a slot of its own; phase A of the target
// block then only sums its slots in a fixed order (deterministic).
//
// Each sweep is one launch. The first kRowSets x kRowWorkers workgroups to
// start are row workers: each owns four point-row slots of every
// kRowSets-th chunk and walks them in chain order, loading its rows' matrix
// slices and taking the part of each row whose inputs are already final
// while the chunk before is still being computed by the other set.
// The other workgroups take the phase A and push items by ticket from a list
// in dependency order, so every item they wait for belongs to a workgroup
// that is already running. Readiness is tracked by counters (per chunk: its
// finished phase A blocks and phase B rows; per target block: its pushed
// entries) compared with multiples of the apply's epoch, polled by one wave
// per workgroup. The one exchange on the chain itself, chunk c-1's rows read
// by the row workers of chunk c, skips the counters: each row result is also
// written as epoch-tagged words that the readers poll directly. The row workers stay resident for the whole launch, so the
// device must hold more workgroups than that at once (checked at setup), and
// sweeps of different streams must not run at the same time (the host orders
// them library-wide). Every wait is bounded: past the context's wait limit it
// gives up, the launch runs to its end and the host reports the timeout.
#include "devcommon.h"
#include "kernels.h"

namespace hs {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / kWave;
constexpr int RB = 16;   // block rows (or rank terms) whose loads are issued together
// the same for blocks of up to Q x 64 points (half as many for Q = 2, so the
// push and phase A registers stay within the row workers' budget)
template <int Q>
constexpr int rb_of() { return Q == 1 ? RB : RB / 2; }

__device__ __forceinline__ int relaxed_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Vectors exchanged between workgroups inside a sweep are read and written
// only with relaxed agent-scope atomics (coherent across the XCDs' L2s by
// themselves), so no cache-wide writeback/invalidate fence is needed; a
// publisher waits for its stores to complete before setting the ready flag.
__device__ __forceinline__ cd ld_sc(const cd* p) {
    const double* d = reinterpret_cast<const double*>(p);
    return cmk(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
               __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_sc(cd* p, cd v) {
    double* d = reinterpret_cast<double*>(p);
    __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Every wait is bounded. Once per kBailPolls polls (every poll when the limit
// is 0) it checks the workspace's error flag and how long it has polled
// (constant-rate device clock); past wk.wait_ticks, or once another wait has
// given up, it sets the flag and returns as if satisfied. The launch then runs to its end on scratch data,
// every later wait of the workspace giving up at its first check, and the
// host turns the flag into an error. The check sits off the poll's fast path,
// so a wait that ends normally costs no extra round trip.
constexpr int kBailPolls = 64;

__device__ __forceinline__ bool must_give_up(const SweepWork& wk, long long t0) {
    return relaxed_load(wk.err) != 0 || wall_clock64() - t0 > wk.wait_ticks;
}
__device__ __forceinline__ void give_up(const SweepWork& wk) {
    __hip_atomic_store(wk.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The chain's critical exchange (chunk c-1's results read by the row workers
// of chunk c) goes through flagged copies: 4 words per complex128 value,
// word w = (epoch << 32) | 32-bit part w of the value. A 64-bit word is
// written and read whole, so a reader that sees the epoch in all four words
// has the value: no store-completion wait, ready count or second load sits
// between the producing row and the row that consumes it.
//
// publish_ll: lane 4 c + w of a wave writes word w of column c of the
// wave-uniform row results y[0 .. cs) of position i.
template <int S>
__device__ __forceinline__ void publish_ll(unsigned long long* ll, int64_t i, int64_t n, int c0, int cs,
                                           const cd (&y)[S], unsigned tag) {
    const int lane = threadIdx.x % kWave;
    const int c = lane / 4, w = lane % 4;
    if (c < cs) {
        cd v = y[0];
#pragma unroll
        for (int cc = 1; cc < S; ++cc)
            if (c == cc) v = y[cc];
        const unsigned long long bits = (unsigned long long)__double_as_longlong(w < 2 ? v.x : v.y);
        const unsigned part = (w & 1) ? (unsigned)(bits >> 32) : (unsigned)bits;
        __hip_atomic_store(ll + ((int64_t)(c0 + c) * n + i) * 4 + w, ((unsigned long long)tag << 32) | part,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// stage_ll: len values per right-hand side (columns c0 .. c0 + cs - 1) from
// position g0 of a flagged copy into LDS x (column stride ld), once every
// word carries tag. Thread t takes words t, t + NT, ... of the contiguous word
// range (a wave's loads cover 512 consecutive bytes) and reloads only the
// words still missing, until no thread of the workgroup misses one. Every
// word is written once per launch by the row worker that owns the position,
// for the same live columns, so the loop ends (or gives up, as the counter
// waits below do).
template <int S>
__device__ __forceinline__ void stage_ll(cd* x, int ld, const unsigned long long* ll, int64_t g0, int len, int64_t n,
                                         int c0, int cs, unsigned tag, const SweepWork& wk) {
    constexpr int PER = (4 * kMaxChunk * S + NT - 1) / NT;
    const int wl = 4 * len, tot = wl * cs;
    unsigned* xw = reinterpret_cast<unsigned*>(x);
    // word e of the range sits at byte 8 (e / wl * 4 n + e % wl) from base
    const char* base = reinterpret_cast<const char*>(ll + ((int64_t)c0 * n + g0) * 4);
    const unsigned cstride = (unsigned)(4 * n);
    unsigned pend = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if ((int)threadIdx.x + u * NT < tot) pend |= 1u << u;
    const long long t0 = wall_clock64();
    for (int round = 1;; ++round) {
        // groups of G words in flight (registers: the row workers hold their
        // matrix rows beside this)
        constexpr int G = 6;
#pragma unroll
        for (int u0 = 0; u0 < PER; u0 += G) {
            unsigned long long w[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                w[u] = 0;
                if (u0 + u < PER && (pend >> (u0 + u) & 1u)) {
                    int e = threadIdx.x + (u0 + u) * NT;
                    asm volatile("" : "+v"(e));   // recomputed per round, not held across the wait
                    const unsigned off = 8u * ((unsigned)(e / wl) * cstride + (unsigned)(e % wl));
                    w[u] = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(base + off), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (u0 + u < PER && (pend >> (u0 + u) & 1u) && (unsigned)(w[u] >> 32) == tag) {
                    const int e = threadIdx.x + (u0 + u) * NT, col = e / wl, r = e % wl;
                    xw[(r / 4 + col * ld) * 4 + r % 4] = (unsigned)w[u];
                    pend &= ~(1u << (u0 + u));
                }
        }
        if (!__syncthreads_or(pend != 0)) break;
        // bounded like the counter waits (one barrier more every kBailPolls rounds)
        if (round % kBailPolls == 0 || wk.wait_ticks == 0) {
            const int bail = threadIdx.x == 0 && must_give_up(wk, t0);
            if (__syncthreads_or(bail)) {
                if (threadIdx.x == 0) give_up(wk);
                break;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __syncthreads();
}

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Loads that write LDS directly (16 bytes per lane: lane l of the wave lands
// at dst + 16 l, dst uniform over the wave), with the same agent-scope
// coherence bit (sc1) as the relaxed agent-scope atomic loads.
__device__ __forceinline__ void load_lds16(const cd* src, cd* dst_wave) {
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                     (__attribute__((address_space(3))) void*)dst_wave, 16, 0, 16);
}

constexpr int PR = (kMaxChunk + NT - 1) / NT;    // r values per thread and column
constexpr int PM = (kFoldCols + NT - 1) / NT;    // early range columns per thread

// Positions of the early range columns l_n + tid + u NT (0 past e_n), loaded
// before the waits (the map is fixed at setup).
__device__ __forceinline__ void load_map(const int32_t* map, int n2, int (&mp)[PM]) {
#pragma unroll
    for (int u = 0; u < PM; ++u) {
        const int k = u * NT + (int)threadIdx.x;
        mp[u] = k < n2 ? map[k] : 0;
    }
}

// Stage r (n1 contiguous values per right-hand side from g1) and the early
// part of the folded range (n2 values per right-hand side gathered from g2 at
// the positions mp) into LDS x1 / x2 (column strides ld1 / ld2). Value k of a
// part is loaded by thread k % NT straight into LDS, so every load of both
// parts is in flight at once and no value passes through registers.
template <int S>
__device__ __forceinline__ void stage_direct(cd* x1, int ld1, const cd* g1, int n1, cd* x2, int ld2, const cd* g2,
                                             const int (&mp)[PM], int n2, int64_t n, int cs) {
    const int tid = threadIdx.x, wb = tid - tid % kWave;
#pragma unroll
    for (int col = 0; col < S; ++col) {
        if (col < cs) {
#pragma unroll
            for (int u = 0; u < PR; ++u) {
                const int k = u * NT + tid;
                if (k < n1) load_lds16(g1 + k + (int64_t)col * n, x1 + col * ld1 + u * NT + wb);
            }
#pragma unroll
            for (int u = 0; u < PM; ++u) {
                const int k = u * NT + tid;
                if (k < n2) load_lds16(g2 + mp[u] + (int64_t)col * n, x2 + col * ld2 + u * NT + wb);
            }
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// v of lane src in every lane (src the same in every lane of the wave)
__device__ __forceinline__ cd bcast_cd(cd v, int src) {
    return cmk(readlane_f64(v.x, src), readlane_f64(v.y, src));
}
__device__ __forceinline__ cd bcast_a(cd v, int src) { return bcast_cd(v, src); }
__device__ __forceinline__ cf bcast_a(cf v, int src) {
    return cmkf(readlane_f32(v.x, src), readlane_f32(v.y, src));
}

__device__ __forceinline__ int take_ticket(unsigned long long* ctr, unsigned long long base, int* s_t) {
    __syncthreads();
    if (threadIdx.x == 0) *s_t = (int)(atomicAdd(ctr, 1ull) - base);
    __syncthreads();
    return *s_t;
}

// Wave-level wait (no fence): counter *cnt == need.
__device__ __forceinline__ void wait_count(const int* cnt, int need, const SweepWork& wk) {
    const long long t0 = wall_clock64();
    for (int it = 1; relaxed_load(cnt) != need; ++it) {
        if ((it % kBailPolls == 0 || wk.wait_ticks == 0) && must_give_up(wk, t0)) {
            give_up(wk);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Three counters polled together (b and c may be null): *a == na, *b == nb
// and *c == nc.
__device__ __forceinline__ void wait_three(const int* a, int na, const int* b, int nb, const int* c, int nc,
                                           const SweepWork& wk) {
    const long long t0 = wall_clock64();
    for (int it = 1;; ++it) {
        const int va = relaxed_load(a);
        const int vb = b ? relaxed_load(b) : nb;
        const int vc = c ? relaxed_load(c) : nc;
        if (va == na && vb == nb && vc == nc) return;
        if ((it % kBailPolls == 0 || wk.wait_ticks == 0) && must_give_up(wk, t0)) {
            give_up(wk);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

constexpr int QC = kMaxChunk / kWave;   // 64-wide column groups of a chunk
constexpr int QF = kFoldCols / kWave;   // column groups of the folded neighbour range

// One row of [A1 | A2] x [x1; x2] by one wave, in parts so that the row's
// loads (independent of the chain) are issued before the wait for its
// inputs: load_row reads A1 (width w1 <= kMaxChunk) and A2 (width w2 <=
// kFoldCols) into registers; row_partial multiplies them with the LDS
// copies of x1 and x2, a column range at a time.
template <class T, class A>
__device__ __forceinline__ void load_row(const T* A1, int w1, const T* A2, int w2, A (&R1)[QC], A (&R2)[QF]) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int q = 0; q < QC; ++q) {
        const int col = lane + q * kWave;
        R1[q] = col < w1 ? to_arith<A>(A1[col]) : czero<A>();
    }
#pragma unroll
    for (int q = 0; q < QF; ++q) {
        const int col = lane + q * kWave;
        R2[q] = col < w2 ? to_arith<A>(A2[col]) : czero<A>();
    }
}

// Lane partial sums of one row (the caller reduces over the wave at the end):
// row_partial takes all of A1 and the A2 columns in [lo, hi); row_head the A2
// columns in [0, hi) with hi <= kMaxChunk, which lie in the first QC groups.
//
// One column: every column group reads LDS at its natural index (inside the
// arrays: xs1 holds kMaxChunk (S + 1) values, see the kernels) and a select
// zeroes the columns outside the row's range, so the reads carry no branch,
// use one base address with immediate offsets and go out XG at a time; the
// exact zeros added leave the sums unchanged. With more columns the
// registers are not there for that, and each group is a guarded read.
template <int S, class A>
__device__ __forceinline__ void row_partial(const A (&R1)[QC], int w1, const cd* xs1, int o1, int ld1,
                                            const A (&R2)[QF], int lo, int hi, const cd* xs2, int ld2, int cs,
                                            A (&acc)[S]) {
    const int lane = threadIdx.x % kWave;
    const A zero = czero<A>();
#pragma unroll
    for (int c = 0; c < S; ++c) {
        if (c < cs) {
            // two interleaved partial sums (even and odd column groups) halve
            // the dependent FMA chain; they are added in a fixed order
            A a[2] = {zero, zero};
            if constexpr (S == 1) {
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int col = lane + q * kWave;
                    const A xv = to_arith<A>(xs1[o1 + col]);
                    a[q & 1] = cfma(R1[q], col < w1 ? xv : zero, a[q & 1]);
                }
                constexpr int XG = 8;
                static_assert(QF % XG == 0, "whole read groups");
#pragma unroll
                for (int q0 = 0; q0 < QF; q0 += XG) {
                    A xv[XG];
#pragma unroll
                    for (int g = 0; g < XG; ++g) xv[g] = to_arith<A>(xs2[lane + (q0 + g) * kWave]);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int g = 0; g < XG; ++g) {
                        const int q = q0 + g, col = lane + q * kWave;
                        a[q & 1] = cfma(R2[q], (col >= lo && col < hi) ? xv[g] : zero, a[q & 1]);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int col = lane + q * kWave;
                    if (col < w1) a[q & 1] = cfma(R1[q], to_arith<A>(xs1[o1 + col + c * ld1]), a[q & 1]);
                }
#pragma unroll
                for (int q = 0; q < QF; ++q) {
                    const int col = lane + q * kWave;
                    if (col >= lo && col < hi) a[q & 1] = cfma(R2[q], to_arith<A>(xs2[col + c * ld2]), a[q & 1]);
                }
            }
            acc[c] = cadd(acc[c], cadd(a[0], a[1]));
        }
    }
}

template <int S, class A>
__device__ __forceinline__ void row_head(const A (&R2)[QF], int hi, const cd* xs2, int ld2, int cs, A (&acc)[S]) {
    const int lane = threadIdx.x % kWave;
    const A zero = czero<A>();
#pragma unroll
    for (int c = 0; c < S; ++c) {
        if (c < cs) {
#pragma unroll
            for (int q = 0; q < QC; ++q) {
                const int col = lane + q * kWave;
                if constexpr (S == 1) {
                    const A xv = to_arith<A>(xs2[col]);
                    acc[c] = cfma(R2[q], col < hi ? xv : zero, acc[c]);
                } else {
                    if (col < hi) acc[c] = cfma(R2[q], to_arith<A>(xs2[col + c * ld2]), acc[c]);
                }
            }
        }
    }
}

// Push of one far entry by one wave. FWD: out[b] = sum_a A[a][b] x[a] with A
// bo x bt (source rows): alpha_kj forward, the transposed copy of a dense
// alpha_kj backward; otherwise out[a] = sum_b A[a][b] x[b] with A = alpha_kj
// (bt x bo, target rows; used for low-rank backward entries). x is the source
// block's segment (elimination order, column stride n); out goes to the
// entry's slot (column stride bt).
template <int S, bool FWD, int Q, class T>
__device__ __forceinline__ void push_one(const PushEnt& e, const T* alpha, const cd* src, int64_t so, int bo, int bt,
                                         int64_t n, int c0, int cs, cd* slot) {
    using A = arith_t<T>;
    const int lane = threadIdx.x % kWave;
    A x[Q][S], acc[Q][S];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int c = 0; c < S; ++c) {
            const int a = lane + q * kWave;
            x[q][c] = (a < bo && c < cs) ? to_arith<A>(ld_sc(src + so + a + (int64_t)(c0 + c) * n)) : czero<A>();
            acc[q][c] = czero<A>();
        }
    const int rows = FWD ? bo : bt, cols = FWD ? bt : bo;
    const T* A_ = alpha + e.aoff;
    if (e.rank < 0) {
        constexpr int RQ = rb_of<Q>();
        for (int a0 = 0; a0 < rows; a0 += RQ) {
            A Ar[RQ][Q];
#pragma unroll
            for (int r = 0; r < RQ; ++r)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int b = lane + q * kWave;
                    Ar[r][q] = (a0 + r < rows && b < cols) ? to_arith<A>(A_[(int64_t)(a0 + r) * cols + b]) : czero<A>();
                }
#pragma unroll
            for (int r = 0; r < RQ; ++r) {
                const int a = a0 + r;
                if (a < rows)
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    if (FWD) {
                        const A xa = bcast_a(a < kWave ? x[0][c] : x[Q - 1][c], a % kWave);
#pragma unroll
                        for (int q = 0; q < Q; ++q) acc[q][c] = cfma(Ar[r][q], xa, acc[q][c]);
                    } else {
                        A sr = cmul(Ar[r][0], x[0][c]);
                        if (Q > 1) sr = cfma(Ar[r][Q - 1], x[Q - 1][c], sr);
                        sr = wave_sum(sr);
                        if (lane == a % kWave) {
                            if (a < kWave) acc[0][c] = cadd(acc[0][c], sr);
                            else acc[Q - 1][c] = cadd(acc[Q - 1][c], sr);
                        }
                    }
                }
            }
        }
    } else {
        const int rk = e.rank;
        const T* Uf = A_;
        const T* Vf = A_ + (int64_t)rows * rk;
        constexpr int RQ = rb_of<Q>();
        for (int l0 = 0; l0 < rk; l0 += RQ) {
            A Ur[RQ][Q], Vr[RQ][Q];
#pragma unroll
            for (int r = 0; r < RQ; ++r)
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int xx = lane + q * kWave;
                    const bool on = l0 + r < rk;
                    Ur[r][q] = (on && xx < rows) ? to_arith<A>(Uf[(int64_t)(l0 + r) * rows + xx]) : czero<A>();
                    Vr[r][q] = (on && xx < cols) ? to_arith<A>(Vf[(int64_t)(l0 + r) * cols + xx]) : czero<A>();
                }
#pragma unroll
            for (int r = 0; r < RQ; ++r) {
                if (l0 + r < rk)
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    if (FWD) {   // V^T (U^T x)
                        A t = cmul(Ur[r][0], x[0][c]);
                        if (Q > 1) t = cfma(Ur[r][Q - 1], x[Q - 1][c], t);
                        t = wave_sum(t);
#pragma unroll
                        for (int q = 0; q < Q; ++q) acc[q][c] = cfma(Vr[r][q], t, acc[q][c]);
                    } else {     // U (V x)
                        A t = cmul(Vr[r][0], x[0][c]);
                        if (Q > 1) t = cfma(Vr[r][Q - 1], x[Q - 1][c], t);
                        t = wave_sum(t);
#pragma unroll
                        for (int q = 0; q < Q; ++q) acc[q][c] = cfma(Ur[r][q], t, acc[q][c]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = lane + q * kWave;
        if (b < bt)
#pragma unroll
            for (int c = 0; c < S; ++c)
                if (c < cs) st_sc(slot + b + (int64_t)c * bt, to_cd(acc[q][c]));
    }
}

// Sum of a target block's slots (fixed order) plus base, one entry per
// thread-owned (row, column) element; base and out in elimination order.
template <int S>
__device__ __forceinline__ void gather_slots(const int64_t* gslot, int64_t g0, int64_t g1, const cd* slots, int nrhs,
                                             int bt, int c0, int cs, const cd* base_lds, cd* out, int64_t n) {
    for (int q = threadIdx.x; q < bt * cs; q += NT) {
        const int a = q % bt, c = q / bt;
        cd s = base_lds[q];
        // GW slot loads in flight per round, added in slot order
        constexpr int GW = 16;
        for (int64_t g = g0; g < g1; g += GW) {
            cd v[GW];
#pragma unroll
            for (int u = 0; u < GW; ++u)
                v[u] = g + u < g1 ? ld_sc(slots + gslot[g + u] * nrhs + (int64_t)(c0 + c) * bt + a) : cmk(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < GW; ++u)
                if (g + u < g1) s = cadd(s, v[u]);
        }
        st_sc(out + a + (int64_t)(c0 + c) * n, s);
    }
}

}  // namespace

// Forward sweep; S right-hand sides per pass.
template <int S, int Q, class T>
__global__ void __launch_bounds__(NT)
k_sweep_fwd(ColMask mk, SweepPlanT<T> p, SweepItems it, const cd* __restrict__ v, SweepWork wk, int nrhs,
            unsigned long long base, int epoch) {
    __shared__ int s_t;
    __shared__ cd bsh[kMaxLeaf * S];
    // xs1 padded by kMaxChunk: the row products read it at o1 + col (< 2 kMaxChunk)
    __shared__ cd xs1[kMaxChunk * (S + 1)];
    __shared__ cd xs2[kFoldCols * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t n = p.n;
    // per-chunk counters one cache line apart (polled by many workgroups)
    int* cntA = wk.flags;
    int* cntB = wk.flags + kCntPad * p.nch;
    int* cntT = wk.flags + 2 * kCntPad * p.nch;
    const int role = take_ticket(wk.tickets, base, &s_t);
    if (role < kRowWorkers * kRowSets) {
        // ---- phase B, persistent: row slot (role % kRowWorkers) * NW + wid of
        // every kRowSets-th chunk in order, y_i = Linv row . r_c + (Linv C) row . y_prev
        const int wkr = role % kRowWorkers;
        const int slot = wkr * NW + wid;
        const int cfirst = role / kRowWorkers;
        if (cfirst >= p.nch) return;
        // the chunk's descriptors and its rows' matrix slices; the next
        // chunk's descriptors are read while this one is in flight, and its
        // rows' loads are issued as soon as this chunk's rows are published
        SweepChunk d = it.fchunk[cfirst];
        RowTask rt = it.frow[d.pc + (slot < d.nc ? slot : 0)];
        arith_t<T> R1[QC], R2[QF];
        int mp[PM];
        load_row(p.lf + rt.a1, slot < d.nc ? rt.w1 : 0, p.mf + rt.a2, slot < d.nc ? d.w2 : 0, R1, R2);
        load_map(it.femap + d.e_off, d.e_n, mp);
        for (int c = cfirst; c < p.nch; c += kRowSets) {
            const bool live = slot < d.nc;
            const int i = d.pc + (live ? slot : 0);
            const int w1 = live ? rt.w1 : 0;
            const int cn = c + kRowSets;
            const SweepChunk dn = it.fchunk[cn < p.nch ? cn : c];
            // phase A of chunk c, and chunks c-2 and c-3 stored and counted: the
            // early range (chunks <= c-2) is then final, since every older
            // chunk's count was awaited by chunk c-2 or c-3 before they ran
            // (chunk c-2 read chunk c-3 from its flagged words, not from its
            // count)
            if (wid == 0)
                wait_three(cntA + kCntPad * c, epoch * d.nblocks, c >= 2 ? cntB + kCntPad * (c - 2) : nullptr,
                           epoch * d.need2, c >= 3 ? cntB + kCntPad * (c - 3) : nullptr, epoch * d.need3, wk);
            __syncthreads();
            compiler_fence();
            bool first = true;   // the first computed pass waits for the newest chunk
            for (int c0 = 0; c0 < nrhs; c0 += S) {
                const int cs = min(S, nrhs - c0);
                if (!cols_live(mk, c0, cs)) continue;
                arith_t<T> acc[S];
#pragma unroll
                for (int cc = 0; cc < S; ++cc) acc[cc] = czero<arith_t<T>>();
                if (first) {
                    // everything but the newest neighbour chunk is final: stage it
                    // and take its part of the row before waiting for that chunk
                    first = false;
                    stage_direct<S>(xs1, d.nc, wk.rbuf + d.pc + (int64_t)c0 * n, d.nc, xs2 + d.l_n, d.w2,
                                    wk.ybuf + (int64_t)c0 * n, mp, d.e_n, n, cs);
                    if (live) row_partial<S>(R1, w1, xs1, rt.o1, d.nc, R2, d.l_n, d.w2, xs2, d.w2, cs, acc);
                    // chunk c-1 (range columns [0, l_n), not read above) as it lands
                    stage_ll<S>(xs2, d.w2, wk.llf, d.l_g, d.l_n, n, c0, cs, (unsigned)epoch, wk);
                    if (live) row_head<S>(R2, d.l_n, xs2, d.w2, cs, acc);
                } else {
                    stage_direct<S>(xs1, d.nc, wk.rbuf + d.pc + (int64_t)c0 * n, d.nc, xs2 + d.l_n, d.w2,
                                    wk.ybuf + (int64_t)c0 * n, mp, d.e_n, n, cs);
                    stage_ll<S>(xs2, d.w2, wk.llf, d.l_g, d.l_n, n, c0, cs, (unsigned)epoch, wk);
                    if (live) {
                        row_partial<S>(R1, w1, xs1, rt.o1, d.nc, R2, d.l_n, d.w2, xs2, d.w2, cs, acc);
                        row_head<S>(R2, d.l_n, xs2, d.w2, cs, acc);
                    }
                }
                if (live) {
                    cd y[S];
#pragma unroll
                    for (int cc = 0; cc < S; ++cc) y[cc] = to_cd(wave_sum(acc[cc]));
                    publish_ll<S>(wk.llf, i, n, c0, cs, y, (unsigned)epoch);
                    if (lane == 0)
#pragma unroll
                        for (int cc = 0; cc < S; ++cc)
                            if (cc < cs) st_sc(wk.ybuf + i + (int64_t)(c0 + cc) * n, y[cc]);
                }
                __syncthreads();
            }
            // one count per workgroup: its live rows, once all of them are stored
            if (live) stores_done();
            __syncthreads();
            const int nlive = min(max(d.nc - wkr * NW, 0), NW);
            if (tid == 0 && nlive > 0)
                __hip_atomic_fetch_add(cntB + kCntPad * c, nlive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cn < p.nch) {
                d = dn;
                rt = it.frow[d.pc + (slot < d.nc ? slot : 0)];
                load_row(p.lf + rt.a1, slot < d.nc ? rt.w1 : 0, p.mf + rt.a2, slot < d.nc ? d.w2 : 0, R1, R2);
                load_map(it.femap + d.e_off, d.e_n, mp);
            }
        }
        return;
    }
    for (int t = role - kRowWorkers * kRowSets;;
         t = take_ticket(wk.tickets, base, &s_t) - kRowWorkers * kRowSets) {
        if (t >= it.nfwd) return;
        const int item = it.fwd[t];
        if (item < p.nb) {
            // ---- phase A: r_j = v_j + sum of the far-entry slots of block j
            const int j = item;
            const int c = p.chunk_of[j];
            const int bj = p.bsize[j];
            const int64_t sj = p.bstart[j], pj = p.pos[j];
            const int nin = (int)(p.fgptr[j + 1] - p.fgptr[j]);
            if (wid == 0 && nin > 0) wait_count(cntT + j, epoch * nin, wk);
            __syncthreads();
            compiler_fence();
            for (int c0 = 0; c0 < nrhs; c0 += S) {
                const int cs = min(S, nrhs - c0);
                if (!cols_live(mk, c0, cs)) continue;
                for (int q = tid; q < bj * cs; q += NT) bsh[q] = v[sj + q % bj + (int64_t)(c0 + q / bj) * n];
                __syncthreads();
                gather_slots<S>(p.fgslot, p.fgptr[j], p.fgptr[j + 1], wk.slots_f, nrhs, bj, c0, cs, bsh, wk.rbuf + pj,
                                n);
                __syncthreads();
            }
            stores_done();
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(cntA + kCntPad * c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // ---- pushes of one source chunk: far entries taken by the waves in turn
            const int g = item - p.nb;
            const int e0 = p.fgrp[g];
            const PushEnt& f0 = p.fpush[e0];
            const int csrc = p.chunk_of[f0.src];
            if (wid == 0) wait_count(cntB + kCntPad * csrc, epoch * p.csize[csrc], wk);
            __syncthreads();
            compiler_fence();
            const int ng = p.fgrp_n[g];
            if (wid < ng) {
                int dst[kPushGroup / NW];
#pragma unroll
                for (int u = 0; u < kPushGroup / NW; ++u) dst[u] = -1;
                for (int q = wid; q < ng; q += NW) {
                    const PushEnt e = p.fpush[e0 + q];
                    dst[q / NW] = e.dst;
                    const int bo = p.bsize[e.src], bt = p.bsize[e.dst];
                    for (int c0 = 0; c0 < nrhs; c0 += S)
                        if (cols_live(mk, c0, min(S, nrhs - c0)))
                            push_one<S, true, Q, T>(e, p.alpha, wk.ybuf, p.pos[e.src], bo, bt, n, c0, min(S, nrhs - c0),
                                                 wk.slots_f + e.slot * nrhs + (int64_t)c0 * bt);
                }
                stores_done();
                if (lane == 0)
#pragma unroll
                    for (int u = 0; u < kPushGroup / NW; ++u)
                        if (dst[u] >= 0) __hip_atomic_fetch_add(cntT + dst[u], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Backward sweep; S right-hand sides per pass.
template <int S, int Q, class T>
__global__ void __launch_bounds__(NT)
k_sweep_bwd(ColMask mk, SweepPlanT<T> p, SweepItems it, cd* __restrict__ z, SweepWork wk, int nrhs,
            unsigned long long base, int epoch, int dmode) {
    __shared__ int s_t;
    __shared__ cd ysh[kMaxLeaf * S];
    __shared__ cd ztsh[kMaxLeaf * S];
    // xs1 padded by kMaxChunk: the row products read it at o1 + col (< 2 kMaxChunk)
    __shared__ cd xs1[kMaxChunk * (S + 1)];
    __shared__ cd xs2[kFoldCols * S];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int64_t n = p.n;
    int* cntA = wk.flags + 2 * kCntPad * p.nch + p.nb;
    int* cntB = wk.flags + 3 * kCntPad * p.nch + p.nb;
    int* cntT = wk.flags + 4 * kCntPad * p.nch + p.nb;
    const int role = take_ticket(wk.tickets + 1, base, &s_t);
    if (role < kRowWorkers * kRowSets) {
        // ---- phase B, persistent: row slot (role % kRowWorkers) * NW + wid of
        // every kRowSets-th chunk, last chunk first,
        // z_i = Linv^T row . r'_c + (Linv^T C') row . z_next
        const int wkr = role % kRowWorkers;
        const int slot = wkr * NW + wid;
        const int cfirst = p.nch - 1 - role / kRowWorkers;
        if (cfirst < 0) return;
        // descriptors and rows fetched one chunk ahead, as in the forward sweep
        SweepChunk d = it.bchunk[cfirst];
        RowTask rt = it.brow[d.pc + (slot < d.nc ? slot : 0)];
        arith_t<T> R1[QC], R2[QF];
        int mp[PM];
        load_row(p.lb + rt.a1, slot < d.nc ? rt.w1 : 0, p.mb + rt.a2, slot < d.nc ? d.w2 : 0, R1, R2);
        load_map(it.bemap + d.e_off, d.e_n, mp);
        for (int c = cfirst; c >= 0; c -= kRowSets) {
            const bool live = slot < d.nc;
            const int i = d.pc + (live ? slot : 0);
            const int w1 = live ? rt.w1 : 0;
            const int cn = c - kRowSets;
            const SweepChunk dn = it.bchunk[cn >= 0 ? cn : c];
            if (wid == 0)   // as in the forward sweep, with chunks c+2 and c+3
                wait_three(cntA + kCntPad * c, epoch * d.nblocks, c + 2 < p.nch ? cntB + kCntPad * (c + 2) : nullptr,
                           epoch * d.need2, c + 3 < p.nch ? cntB + kCntPad * (c + 3) : nullptr, epoch * d.need3, wk);
            __syncthreads();
            compiler_fence();
            bool first = true;   // the first computed pass waits for the newest chunk
            for (int c0 = 0; c0 < nrhs; c0 += S) {
                const int cs = min(S, nrhs - c0);
                if (!cols_live(mk, c0, cs)) continue;
                arith_t<T> acc[S];
#pragma unroll
                for (int cc = 0; cc < S; ++cc) acc[cc] = czero<arith_t<T>>();
                if (first) {
                    // everything but the newest neighbour chunk is final: stage it
                    // and take its part of the row before waiting for that chunk
                    first = false;
                    stage_direct<S>(xs1, d.nc, wk.rbuf2 + d.pc + (int64_t)c0 * n, d.nc, xs2 + d.l_n, d.w2,
                                    wk.zbuf + (int64_t)c0 * n, mp, d.e_n, n, cs);
                    if (live) row_partial<S>(R1, w1, xs1, rt.o1, d.nc, R2, d.l_n, d.w2, xs2, d.w2, cs, acc);
                    // chunk c+1 (range columns [0, l_n), not read above) as it lands
                    stage_ll<S>(xs2, d.w2, wk.llb, d.l_g, d.l_n, n, c0, cs, (unsigned)epoch, wk);
                    if (live) row_head<S>(R2, d.l_n, xs2, d.w2, cs, acc);
                } else {
                    stage_direct<S>(xs1, d.nc, wk.rbuf2 + d.pc + (int64_t)c0 * n, d.nc, xs2 + d.l_n, d.w2,
                                    wk.zbuf + (int64_t)c0 * n, mp, d.e_n, n, cs);
                    stage_ll<S>(xs2, d.w2, wk.llb, d.l_g, d.l_n, n, c0, cs, (unsigned)epoch, wk);
                    if (live) {
                        row_partial<S>(R1, w1, xs1, rt.o1, d.nc, R2, d.l_n, d.w2, xs2, d.w2, cs, acc);
                        row_head<S>(R2, d.l_n, xs2, d.w2, cs, acc);
                    }
                }
                if (live) {
                    cd y[S];
#pragma unroll
                    for (int cc = 0; cc < S; ++cc) y[cc] = to_cd(wave_sum(acc[cc]));
                    publish_ll<S>(wk.llb, i, n, c0, cs, y, (unsigned)epoch);
                    if (lane == 0)
#pragma unroll
                        for (int cc = 0; cc < S; ++cc)
                            if (cc < cs) {
                                st_sc(wk.zbuf + i + (int64_t)(c0 + cc) * n, y[cc]);
                                z[rt.zpos + (int64_t)(c0 + cc) * n] = y[cc];
                            }
                }
                __syncthreads();
            }
            // one count per workgroup: its live rows, once all of them are stored
            if (live) stores_done();
            __syncthreads();
            const int nlive = min(max(d.nc - wkr * NW, 0), NW);
            if (tid == 0 && nlive > 0)
                __hip_atomic_fetch_add(cntB + kCntPad * c, nlive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cn >= 0) {
                d = dn;
                rt = it.brow[d.pc + (slot < d.nc ? slot : 0)];
                load_row(p.lb + rt.a1, slot < d.nc ? rt.w1 : 0, p.mb + rt.a2, slot < d.nc ? d.w2 : 0, R1, R2);
                load_map(it.bemap + d.e_off, d.e_n, mp);
            }
        }
        return;
    }
    for (int t = role - kRowWorkers * kRowSets;;
         t = take_ticket(wk.tickets + 1, base, &s_t) - kRowWorkers * kRowSets) {
        if (t >= it.nbwd) return;
        const int item = it.bwd[t];
        if (item < p.nb) {
            // ---- phase A: r'_k = D_k^-1 y_k + sum of the far-entry slots of block k
            const int k = item;
            const int c = p.chunk_of[k];
            const int bk = p.bsize[k];
            const int64_t pk = p.pos[k];
            const T* Di = p.dinv + p.dinv_off[k];
            const int nin = (int)(p.bgptr[k + 1] - p.bgptr[k]);
            if (wid == 0 && nin > 0) wait_count(cntT + k, epoch * nin, wk);
            __syncthreads();
            compiler_fence();
            for (int c0 = 0; c0 < nrhs; c0 += S) {
                const int cs = min(S, nrhs - c0);
                if (!cols_live(mk, c0, cs)) continue;
                for (int q = tid; q < bk * cs; q += NT) ysh[q] = wk.ybuf[pk + q % bk + (int64_t)(c0 + q / bk) * n];
                __syncthreads();
                constexpr int RQ = rb_of<Q>();
                if (!dmode)   // alpha alone (no block-diagonal solve): r'_k = y_k + slots
                    for (int q = tid; q < bk * cs; q += NT) ztsh[q] = ysh[q];
                for (int a0 = dmode ? wid : bk; a0 < bk; a0 += NW * RQ) {
                    cd Dr[RQ][Q];
#pragma unroll
                    for (int r = 0; r < RQ; ++r)
#pragma unroll
                        for (int q = 0; q < Q; ++q) {
                            const int aa = a0 + NW * r, b = lane + q * kWave;
                            Dr[r][q] = (aa < bk && b < bk) ? to_cd(Di[(int64_t)aa * bk + b]) : cmk(0.0, 0.0);
                        }
#pragma unroll
                    for (int r = 0; r < RQ; ++r) {
                        const int aa = a0 + NW * r;
                        if (aa < bk)
#pragma unroll
                        for (int cc = 0; cc < S; ++cc) {
                            cd sacc = cmk(0.0, 0.0);
#pragma unroll
                            for (int q = 0; q < Q; ++q) {
                                const int b = lane + q * kWave;
                                if (b < bk) sacc = cfma(Dr[r][q], ysh[b + cc * bk], sacc);
                            }
                            sacc = wave_sum(sacc);
                            if (lane == 0 && cc < cs) ztsh[aa + cc * bk] = sacc;
                        }
                    }
                }
                __syncthreads();
                gather_slots<S>(p.bgslot, p.bgptr[k], p.bgptr[k + 1], wk.slots_b, nrhs, bk, c0, cs, ztsh, wk.rbuf2 + pk,
                                n);
                __syncthreads();
            }
            stores_done();
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(cntA + kCntPad * c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // ---- pushes of one source chunk: alpha_kj z_j into the slot of (k, j)
            const int g = item - p.nb;
            const int e0 = p.bgrp[g];
            const PushEnt& b0 = p.bpush[e0];
            const int csrc = p.chunk_of[b0.src];
            if (wid == 0) wait_count(cntB + kCntPad * csrc, epoch * p.csize[csrc], wk);
            __syncthreads();
            compiler_fence();
            const int ng = p.bgrp_n[g];
            if (wid < ng) {
                int dst[kPushGroup / NW];
#pragma unroll
                for (int u = 0; u < kPushGroup / NW; ++u) dst[u] = -1;
                for (int q = wid; q < ng; q += NW) {
                    const PushEnt e = p.bpush[e0 + q];
                    dst[q / NW] = e.dst;
                    const int bo = p.bsize[e.src], bt = p.bsize[e.dst];
                    for (int c0 = 0; c0 < nrhs; c0 += S) {
                        if (!cols_live(mk, c0, min(S, nrhs - c0))) continue;
                        cd* slot = wk.slots_b + e.slot * nrhs + (int64_t)c0 * bt;
                        if (e.rank < 0)   // column sums over the transposed copy
                            push_one<S, true, Q, T>(e, p.alpha_t, wk.zbuf, p.pos[e.src], bo, bt, n, c0,
                                                 min(S, nrhs - c0), slot);
                        else
                            push_one<S, false, Q, T>(e, p.alpha, wk.zbuf, p.pos[e.src], bo, bt, n, c0,
                                                  min(S, nrhs - c0), slot);
                    }
                }
                stores_done();
                if (lane == 0)
#pragma unroll
                    for (int u = 0; u < kPushGroup / NW; ++u)
                        if (dst[u] >= 0) __hip_atomic_fetch_add(cntT + dst[u], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// Linv rows of each chunk, row blocks in order:
// X_j = E_j + sum_{in-chunk (k, j)} alpha_kj^T X_k, X_k stored b_k x w_k.
// Columns are independent, so each workgroup takes a slice of kLinvCols
// columns of one chunk and keeps that slice of the chunk's rows in LDS.
constexpr int kLinvCols = 8;
__global__ void __launch_bounds__(NT)
k_linv(SweepPlan p, const int32_t* __restrict__ chunk_first, const int64_t* __restrict__ intptr,
       const SweepEnt* __restrict__ intent, const cd* __restrict__ A, cd* __restrict__ lf) {
    constexpr int NS = kMaxChunk / kLinvCols;
    const int c = blockIdx.x / NS;
    const int col0 = (blockIdx.x % NS) * kLinvCols;
    if (col0 >= p.csize[c]) return;
    __shared__ cd Xs[kMaxChunk][kLinvCols];
    const int j0 = chunk_first[c], j1 = chunk_first[c + 1];
    for (int j = j0; j < j1; ++j) {
        const int bj = p.bsize[j], wj = p.w[j], lj = p.loc[j];
        cd* X = lf + p.lf_off[j];
        for (int e = threadIdx.x; e < bj * kLinvCols; e += NT) {
            const int a = e / kLinvCols, cl = e % kLinvCols, col = col0 + cl;
            if (col >= wj) continue;
            cd val = cmk(col == lj + a ? 1.0 : 0.0, 0.0);
            for (int64_t q = intptr[j]; q < intptr[j + 1]; ++q) {
                const SweepEnt en = intent[q];
                const int k = en.k, bk = p.bsize[k], lk = p.loc[k];
                if (col >= p.w[k]) continue;
                const cd* Ak = A + en.off;
                for (int l = 0; l < bk; ++l) val = cfma(Ak[(int64_t)l * bj + a], Xs[lk + l][cl], val);
            }
            Xs[lj + a][cl] = val;
            X[(int64_t)a * wj + col] = val;
        }
        __syncthreads();
    }
}

// Linv^T row block k: LT_k[a][col] = Linv[loc_k + col][loc_k + a], col < wt_k.
__global__ void __launch_bounds__(NT)
k_linv_transpose(SweepPlan p, cd* __restrict__ lb) {
    const int k = blockIdx.x;
    const int bk = p.bsize[k], wtk = p.wt[k], lk = p.loc[k];
    const int cl = p.clast[k];
    cd* out = lb + p.lb_off[k];
    for (int e = threadIdx.x; e < bk * wtk; e += NT) {
        const int a = e / wtk, col = e % wtk;
        const int row = lk + col;          // chunk row index
        // find the block kp holding chunk row `row` (blocks k..cl)
        int kp = k;
        while (kp < cl && p.loc[kp] + p.bsize[kp] <= row) ++kp;
        const int rr = row - p.loc[kp];
        const int wkp = p.w[kp];
        const int cc = lk + a;
        out[e] = cc < wkp ? p.lf[p.lf_off[kp] + (int64_t)rr * wkp + cc] : cmk(0.0, 0.0);
    }
}

__global__ void __launch_bounds__(NT)
k_lr_expand(const ExpandTask* __restrict__ tasks, const cd* __restrict__ src, cd* __restrict__ dst) {
    const ExpandTask t = tasks[blockIdx.x];
    const cd* U = src + t.src_off;
    const cd* V = U + (int64_t)t.m * t.r;
    cd* D = dst + t.dst_off;
    for (int e = threadIdx.x; e < t.m * t.n; e += NT) {
        const int a = e / t.n, b = e % t.n;
        cd s = cmk(0.0, 0.0);
        for (int l = 0; l < t.r; ++l) s = cfma(U[(int64_t)l * t.m + a], V[(int64_t)l * t.n + b], s);
        D[e] = s;
    }
}

int sweep_grid(int64_t nitems) {
    constexpr int rows = kRowWorkers * kRowSets;
    const int64_t others = nitems < 1 ? 1 : (nitems < 1024 - rows ? nitems : 1024 - rows);
    return rows + (int)others;
}

int sweep_capacity(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    int mn = 1 << 30;
    auto chk = [&](const void* f) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f, NT, 0) != hipSuccess) b = 0;
        mn = b < mn ? b : mn;
    };
#define HS_CHK(SS, QQ, TT)                                                     \
    chk(reinterpret_cast<const void*>(&k_sweep_fwd<SS, QQ, TT>));              \
    chk(reinterpret_cast<const void*>(&k_sweep_bwd<SS, QQ, TT>))
    HS_CHK(1, 1, cd);
    HS_CHK(1, 2, cd);
    HS_CHK(2, 1, cd);
    HS_CHK(2, 2, cd);
    HS_CHK(1, 1, cf);
    HS_CHK(1, 2, cf);
    HS_CHK(2, 1, cf);
    HS_CHK(2, 2, cf);
#undef HS_CHK
    return mn * cus;
}

namespace {
template <class T>
void sweep(bool forward, const ColMask& mk, const SweepPlanT<T>& p, const SweepItems& it, const cd* v, cd* z, int nrhs,
           const SweepWork& w, int epoch, bool dinv, hipStream_t s) {
    const int64_t nit = forward ? it.nfwd : it.nbwd;
    const int G = sweep_grid(nit);
    const unsigned long long base = (unsigned long long)(epoch - 1) * (unsigned long long)(nit + G);
    const bool wide = p.bmax > kWave;
#define HS_SWEEP(SS, QQ)                                                                                          \
    do {                                                                                                           \
        if (forward)                                                                                               \
            hipLaunchKernelGGL((k_sweep_fwd<SS, QQ, T>), dim3(G), dim3(NT), 0, s, mk, p, it, v, w, nrhs, base, epoch); \
        else                                                                                                       \
            hipLaunchKernelGGL((k_sweep_bwd<SS, QQ, T>), dim3(G), dim3(NT), 0, s, mk, p, it, z, w, nrhs, base, epoch, \
                               (int)dinv);                                                                     \
    } while (0)
    if (nrhs == 1) {
        if (wide) HS_SWEEP(1, 2); else HS_SWEEP(1, 1);
    } else {
        if (wide) HS_SWEEP(2, 2); else HS_SWEEP(2, 1);
    }
#undef HS_SWEEP
}
}  // namespace

void launch_sweep(bool forward, const ColMask& mk, const SweepPlan& p, const SweepItems& it, const cd* v, cd* z,
                  int nrhs, const SweepWork& w, int epoch, hipStream_t s, bool dinv) {
    sweep(forward, mk, p, it, v, z, nrhs, w, epoch, dinv, s);
}
void launch_sweep(bool forward, const ColMask& mk, const SweepPlanT<cf>& p, const SweepItems& it, const cd* v, cd* z,
                  int nrhs, const SweepWork& w, int epoch, hipStream_t s, bool dinv) {
    sweep(forward, mk, p, it, v, z, nrhs, w, epoch, dinv, s);
}

// Vectors between tree order and the sweeps' elimination-order work buffer
// (block k at pos[k]); N x nrhs, column stride n in both.
__global__ void k_elim_move(SweepPlan p, const cd* __restrict__ src, cd* __restrict__ dst, int nrhs, int to_elim) {
    const int k = blockIdx.x, c = blockIdx.y;
    const int bk = p.bsize[k];
    const int64_t t0 = p.bstart[k] + (int64_t)c * p.n, e0 = p.pos[k] + (int64_t)c * p.n;
    for (int a = threadIdx.x; a < bk; a += blockDim.x) {
        if (to_elim) dst[e0 + a] = src[t0 + a];
        else dst[t0 + a] = src[e0 + a];
    }
}

// out = add + D^-1 in block by block (add may be null), tree order; one
// workgroup per block and column, one wave per row of D_k^-1.
__global__ void __launch_bounds__(NT) k_block_dinv(SweepPlan p, const cd* __restrict__ in, const cd* __restrict__ add,
                                                   cd* __restrict__ out, int nrhs) {
    const int k = blockIdx.x, c = blockIdx.y;
    const int bk = p.bsize[k];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int64_t t0 = p.bstart[k] + (int64_t)c * p.n;
    const cd* Di = p.dinv + p.dinv_off[k];
    for (int a = wid; a < bk; a += NW) {
        cd s = cmk(0.0, 0.0);
        for (int b = lane; b < bk; b += kWave) s = cfma(Di[(int64_t)a * bk + b], in[t0 + b], s);
        s = wave_sum(s);
        if (lane == 0) out[t0 + a] = add ? cadd(add[t0 + a], s) : s;
    }
}

void launch_elim_move(const SweepPlan& p, const cd* src, cd* dst, int nrhs, bool to_elim, hipStream_t s) {
    if (p.nb > 0)
        hipLaunchKernelGGL(k_elim_move, dim3(p.nb, nrhs), dim3(64), 0, s, p, src, dst, nrhs, (int)to_elim);
}

void launch_block_dinv(const SweepPlan& p, const cd* in, const cd* add, cd* out, int nrhs, hipStream_t s) {
    if (p.nb > 0) hipLaunchKernelGGL(k_block_dinv, dim3(p.nb, nrhs), dim3(NT), 0, s, p, in, add, out, nrhs);
}

void launch_linv(const SweepPlan& p, int nchunk, const int32_t* chunk_first, const int64_t* intptr,
                 const SweepEnt* intent, const cd* A, cd* lf, hipStream_t s) {
    if (nchunk > 0)
        hipLaunchKernelGGL(k_linv, dim3((unsigned)nchunk * (kMaxChunk / kLinvCols)), dim3(NT), 0, s, p, chunk_first,
                           intptr, intent, A, lf);
}

void launch_linv_transpose(const SweepPlan& p, cd* lb, hipStream_t s) {
    if (p.nb > 0) hipLaunchKernelGGL(k_linv_transpose, dim3(p.nb), dim3(NT), 0, s, p, lb);
}

void launch_lr_expand(const ExpandTask* tasks, int64_t ntasks, const cd* src, cd* dst, hipStream_t s) {
    if (ntasks > 0) hipLaunchKernelGGL(k_lr_expand, dim3((unsigned)ntasks), dim3(NT), 0, s, tasks, src, dst);
}

}  // namespace hs
