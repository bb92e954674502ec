// Internal definitions shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tfft {

// Pass roles of the tiled FFT (TurboFFT Section IV-A.1).  A length-N signal
// is split N = M_1 * ... * M_P (P <= 3); pass p transforms axis p.
//  ROWS     one-pass plan: each signal is contiguous, output contiguous.
//  STRIDED  pass p < P: within each block of L_p = M_p * ... * M_P elements,
//           the M_p elements of axis p are S_p = L_p / M_p apart; the result
//           is multiplied by the twiddle w_{L_p}^{k_p i} (i = position inside
//           the stride) and stored back in place, in the same layout.
//  LAST     pass P: contiguous rows of length M_P; the outputs are stored
//           transposed, y[r + (N / M_P) k_P], r the digit-reversed row.
enum Kind { KIND_ROWS = 0, KIND_STRIDED = 1, KIND_LAST = 2 };
constexpr int kMaxPasses = 3;

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
constexpr int ipowc(int b, int e) { return e == 0 ? 1 : b * ipowc(b, e - 1); }

// ---------------------------------------------------------------- config
// Compile-time configuration (values measured on MI355X; -D overrides them).
#ifndef TFFT_E32
#define TFFT_E32 8
#endif
#ifndef TFFT_E64
#define TFFT_E64 8
#endif
// Elements held by one thread (the thread-level radix, Section IV-A.2);
// complex128 transforms of at least TFFT_E64_BIG_MIN points may use a larger
// thread radix (fewer stages and threads per signal).
#ifndef TFFT_E64_BIG
#define TFFT_E64_BIG TFFT_E64
#endif
#ifndef TFFT_E64_BIG_MIN
#define TFFT_E64_BIG_MIN 4096
#endif
// complex64 strided / last passes of at least TFFT_E32_MP_BIG_MIN points may
// use a larger thread radix, so that their tiles keep >= 16 columns (128-byte
// rows) within 512 threads.
#ifndef TFFT_E32_MP_BIG
#define TFFT_E32_MP_BIG TFFT_E32
#endif
#ifndef TFFT_E32_MP_BIG_MIN
#define TFFT_E32_MP_BIG_MIN 512
#endif
// Occupancy floor of the pass kernels (waves per SIMD the compiler must
// allow, which caps the registers per thread); 0 = the compiler's choice.
#ifndef TFFT_WAVES_PER_EU
#define TFFT_WAVES_PER_EU 0
#endif
// One-pass tiles of at least TFFT_E_ROWS_BIG_MIN points use a thread radix
// of TFFT_E_ROWS_BIG (fewer, larger threads: 512 threads of 16 points for 8192
// points keep 256 VGPRs per thread where 1024 threads of 8 would spill).
#ifndef TFFT_E_ROWS_BIG
#define TFFT_E_ROWS_BIG 16
#endif
#ifndef TFFT_E_ROWS_BIG_MIN
#define TFFT_E_ROWS_BIG_MIN 8192
#endif
constexpr int cfg_E(int fp64, int M, int kind) {
    const int e = (kind == KIND_ROWS && M >= TFFT_E_ROWS_BIG_MIN)
                      ? TFFT_E_ROWS_BIG
                      : fp64 ? (M >= TFFT_E64_BIG_MIN ? TFFT_E64_BIG : TFFT_E64)
                             : ((kind != KIND_ROWS && M >= TFFT_E32_MP_BIG_MIN) ? TFFT_E32_MP_BIG : TFFT_E32);
    return M >= e ? e : M;
}
// Threads of a multi-pass tile (a 512-thread workgroup caps a wavefront at
// 256 VGPRs, a 256-thread one lets the compiler use the accumulation
// registers as well).
#ifndef TFFT_MP_THREADS32
#define TFFT_MP_THREADS32 512
#endif
#ifndef TFFT_MP_THREADS64
#define TFFT_MP_THREADS64 512
#endif
// Signals held in LDS at once by one workgroup (the tile).  One-pass tiles
// aim at 256 threads; multi-pass tiles are as wide as 512 threads and 64 KiB
// of LDS allow (at most 32 signals), because the strided loads and the
// transposed stores of those passes move C adjacent elements per row.
constexpr int cfg_C(int fp64, int M, int kind) {
    const int E = cfg_E(fp64, M, kind);
    const int T = M / E;
    const int S = fp64 ? 16 : 8;
    int c = kind == KIND_ROWS ? 256 / (T > 0 ? T : 1) : 32;
    if (kind == KIND_ROWS && c > 16) c = 16;
    const int maxthr = kind == KIND_ROWS ? 256 : (fp64 ? TFFT_MP_THREADS64 : TFFT_MP_THREADS32);
    while (c > 1 && (c * T > maxthr || c * M * S > 65536)) c /= 2;
    return c < 1 ? 1 : c;
}
// Keep the stage twiddles / the checksum vector of a thread in registers
// across the signals it processes (1), or re-read them from the L1/L2
// resident tables for every signal (0).
#ifndef TFFT_TWREG32
#define TFFT_TWREG32 1
#endif
#ifndef TFFT_TWREG64
#define TFFT_TWREG64 0
#endif
#ifndef TFFT_CREG32
#define TFFT_CREG32 1
#endif
// Stage twiddles not kept in registers come from an LDS octant table (1) or
// from the L1/L2-resident global table (0); LDS-prefetching kernels always
// use the LDS table.
#ifndef TFFT_TWLDS
#define TFFT_TWLDS 0
#endif
#ifndef TFFT_CREG64
#define TFFT_CREG64 0
#endif
#ifndef TFFT_PREFETCH32
#define TFFT_PREFETCH32 1
#endif
#ifndef TFFT_PREFETCH64
#define TFFT_PREFETCH64 0
#endif
// Workgroups per launch: this many times the resident capacity of the chip
// (0: at most 2048).
#ifndef TFFT_GRID_MULT
#define TFFT_GRID_MULT 0
#endif
// Streaming (non-temporal) global loads and stores of the signal data;
// multi-pass tiles with rows narrower than TFFT_NT_MIN_ROW bytes store
// through the cache.
#ifndef TFFT_NT
#define TFFT_NT 1
#endif
#ifndef TFFT_NT_MIN_ROW
#define TFFT_NT_MIN_ROW 128
#endif
// Member addressing of multi-pass tiles by shifts and masks (1) or by 64-bit
// divisions (0); n_strips and O are powers of two.
#ifndef TFFT_MEMBER_SHIFT
#define TFFT_MEMBER_SHIFT 0
#endif
// Strided passes (whose outputs the next pass reads) store streaming (1) or
// through the caches (0).
#ifndef TFFT_NT_STRIDED_ST
#define TFFT_NT_STRIDED_ST 1
#endif
// Total threads of one launch when it is not persistent (workgroups capped
// at this divided by the workgroup size).
#ifndef TFFT_GRID_THREADS
#define TFFT_GRID_THREADS (4096 * 256)
#endif
// Multi-pass kernels of at least this many points per sub-transform get
// twice that many workgroups (measured: complex64 N = 2^18 and 2^19 7-8%
// faster, complex128 neutral; the shorter multi-pass tiles lose with it).
// 0 = off.
#ifndef TFFT_GRID_MP_BIG_M
#define TFFT_GRID_MP_BIG_M 512
#endif
// Largest log2(N) planned with two passes (three passes above), per element
// type (measured: complex64 N = 2^20 as 1024 x 1024 has 32-byte tile rows in
// its first pass and is faster in three).
#ifndef TFFT_TWO_PASS_MAX_LOG2_32
#define TFFT_TWO_PASS_MAX_LOG2_32 19
#endif
#ifndef TFFT_TWO_PASS_MAX_LOG2_64
#define TFFT_TWO_PASS_MAX_LOG2_64 20
#endif
// Default threshold factors kappa, calibrated on >= 10^6 fault-free groups
// per precision (N(0,1) and six-decade lognormal inputs, N = 2^8..2^24): the
// largest noise-scaled residual |d1| / (tau / kappa) was 8.4 for complex64
// and 47 for complex128, whose checksum arithmetic (binary64) rounds as
// coarsely as its data.
#ifndef TFFT_KAPPA32
#define TFFT_KAPPA32 16.0
#endif
#ifndef TFFT_KAPPA64
#define TFFT_KAPPA64 96.0
#endif
// Workgroups (of 512 threads) of the streaming copy instrument (measured:
// 16384 workgroups of 512 threads, four 16-byte elements in flight per
// thread, reach the highest copy bandwidth).
#ifndef TFFT_COPY_GRID
#define TFFT_COPY_GRID 16384
#endif
// Parallel branches of a captured ragged graph (independent length classes).
#ifndef TFFT_GRAPH_BRANCHES
#define TFFT_GRAPH_BRANCHES 4
#endif
// One-pass plans up to 2^TFFT_ONE_PASS_MAX_LOG2 points (the tile of one
// signal: 64 KiB complex64, 128 KiB complex128 of LDS).
#ifndef TFFT_ONE_PASS_MAX_LOG2
#define TFFT_ONE_PASS_MAX_LOG2 12
#endif
// Lengths from which a thread keeps no stage twiddles and no checksum vector
// in registers (1024-thread one-pass tiles: 128 VGPRs per thread); their
// stage twiddles come from the LDS octant table.
#ifndef TFFT_BIG_ROWS_M
#define TFFT_BIG_ROWS_M 8192
#endif
constexpr int cfg_twreg(int fp64, int M, int kind) { return M >= TFFT_BIG_ROWS_M ? 0 : (fp64 ? TFFT_TWREG64 : TFFT_TWREG32); }
constexpr int cfg_creg(int fp64, int M, int kind) { return M >= TFFT_BIG_ROWS_M ? 0 : (fp64 ? TFFT_CREG64 : TFFT_CREG32); }
constexpr int cfg_twlds(int fp64, int M, int kind) { return TFFT_TWLDS || M >= TFFT_BIG_ROWS_M; }
// Issue the next tile's loads before transforming the current one (the
// complex128 tiles that cannot double-buffer in LDS prefetch into registers).
#ifndef TFFT_PREFETCH64_BIG
#define TFFT_PREFETCH64_BIG 1
#endif
constexpr int cfg_prefetch(int fp64, int M, int kind) {
    return fp64 ? (TFFT_PREFETCH64 || (TFFT_PREFETCH64_BIG && M >= TFFT_BIG_ROWS_M)) : TFFT_PREFETCH32;
}
// Correction launch: at most TFFT_CORRECT_GRID workgroups (one per record,
// the rest exit at once), each summing group members TFFT_CORRECT_BATCH at a
// time.
#ifndef TFFT_CORRECT_GRID
#define TFFT_CORRECT_GRID 1024
#endif
#ifndef TFFT_CORRECT_BATCH
#define TFFT_CORRECT_BATCH 8
#endif
// Group sums of the two-sided checksum reduced through LDS by one wavefront
// (1) or by DPP in every wavefront (0; measured faster: the LDS variant's two
// extra barriers per group cost more than the DPP instructions it saves).
#ifndef TFFT_LDS_RED
#define TFFT_LDS_RED 0
#endif
// The decision of a group taken one group later (1), from partial sums kept
// in a second LDS slot, so that the group's end needs no barrier of its own
// (the next group's exchange barriers order the partial sums' writes and
// reads), or at the group's end between two barriers (0).
#ifndef TFFT_RED_DEFER
#define TFFT_RED_DEFER 1
#endif
// Deferred stores (see the pass kernel): 0 never, 1 in LDS-prefetching
// one-pass kernels, 2 in every prefetching kernel (measured: 2-8% slower on
// the multi-pass sizes, where the kept registers cost more than the wait).
#ifndef TFFT_DEFER_ST
#define TFFT_DEFER_ST 1
#endif
constexpr bool cfg_defer(int fp64, int M, int kind) {
    return TFFT_DEFER_ST == 2 || (TFFT_DEFER_ST == 1 && fp64 && kind == KIND_ROWS);
}
// Order the register prefetch after the current tile's values are in
// registers, with branch-free tile loads (see the pass kernel): multi-pass
// tiles, and one-pass tiles of at least TFFT_PF_FENCE_ROWS_MIN points
// (measured: faster there, slower for the short one-pass sizes).
#ifndef TFFT_PF_FENCE
#define TFFT_PF_FENCE 1
#endif
#ifndef TFFT_PF_FENCE_ROWS_MIN
#define TFFT_PF_FENCE_ROWS_MIN 4096
#endif
constexpr int cfg_pf_fence(int fp64, int M, int kind) {
    return TFFT_PF_FENCE && (kind != KIND_ROWS || M >= TFFT_PF_FENCE_ROWS_MIN) ? 1 : 0;
}
constexpr int cfg_threads(int fp64, int M, int kind) { return cfg_C(fp64, M, kind) * (M / cfg_E(fp64, M, kind)); }
// Prefetch of the next tile straight into a second LDS buffer
// (global_load_lds_dwordx4: 16-byte elements, i.e. complex128) for tiles of
// at least TFFT_LDSPF64_MIN points whose two buffers fit in 128 KiB and
// whose workgroup is whole wavefronts.  TFFT_LDSPF64: 0 off, 1 one-pass
// tiles only, 2 all kinds.
#ifndef TFFT_LDSPF64
#define TFFT_LDSPF64 2
#endif
#ifndef TFFT_LDSPF64_MIN
#define TFFT_LDSPF64_MIN 16
#endif
constexpr int cfg_ldspf(int fp64, int M, int kind) {
    return (fp64 && (TFFT_LDSPF64 == 2 || (TFFT_LDSPF64 == 1 && kind == KIND_ROWS)) && M >= TFFT_LDSPF64_MIN &&
            cfg_C(fp64, M, kind) * M * 16 * 2 <= 131072 && cfg_threads(fp64, M, kind) % 64 == 0)
               ? 1
               : 0;
}

// Radix sequence: as many stages of radix E as fit, then one stage of the
// remaining factor (which divides E).
constexpr int n_full(int M, int E) { return E <= 1 ? 0 : ilog2c(M) / ilog2c(E); }
constexpr int n_stages(int M, int E) { return ipowc(E, n_full(M, E)) == M ? n_full(M, E) : n_full(M, E) + 1; }
constexpr int stage_radix(int M, int E, int s) { return s < n_full(M, E) ? E : M / ipowc(E, n_full(M, E)); }
constexpr int stage_ns(int M, int E, int s) { return s <= n_full(M, E) ? ipowc(E, s) : M; }

// ---------------------------------------------------------------- report
struct DevRecord {
    int64_t group;
    int32_t pass, action, member, method;
    int32_t task, pad_;  // persistent ragged kernel: the (class, pass) task; 0 otherwise
    double d1r, d1i, d2r, d2i, tau, s;
};

struct DevReport {
    unsigned long long n_flag;         // flagged groups (record slots requested)
    unsigned long long corrected, benign, uncorrectable;
};

// One fault, resolved by the host to the register that holds the element.
struct DevFault {
    int64_t group;   // group within the pass
    int32_t member;  // member within the group
    int32_t stage;   // butterfly stage, -1 = final value
    int32_t j, m;    // thread within the signal, register index
    int32_t next;    // next fault of the same group, -1 = end
    int32_t mode;    // 0 add, 1 flip a bit of re, 2 flip a bit of im
    double dre, dim;
    int32_t bit;
    int32_t pad_;
};

// Geometry and tables of one pass launch.
struct PassArgs {
    const void *in;
    void *out;
    int64_t batch;      // B
    int64_t n;          // full transform length N
    int64_t L;          // STRIDED: block length L_p
    int32_t S;          // STRIDED: stride S_p of the transform axis
    int32_t O;          // STRIDED: blocks per signal (N / L_p)
    int64_t rows;       // LAST: rows per signal, N / M_P (output stride)
    int32_t m1, m2;     // LAST: row r comes from block (r mod m1) * m2 + r / m1
    int32_t G;          // members per checksum group
    int32_t rb;         // multi-pass: outer units per group (G = C * rb)
    int64_t n_strips;   // multi-pass: tiles of C sub-signals per outer unit
    int64_t n_outer;    // multi-pass: outer units (B * O for STRIDED, B for LAST)
    int64_t n_groups;   // groups of this launch
    int64_t tw_scale;   // STRIDED: w_{L}^t = w_N^{t * tw_scale}
    int32_t conj_in, conj_out;
    double out_scale;   // applied to the final values when != 1
    const double *cvec; // [2M] checksum vector c of this pass and direction (fp64)
    const void *stw;    // [2M] stage twiddles w_M^t in the element type
    const double *stw64;// [2M] the same in fp64 (correction path)
    const double *itw_lo, *itw_hi; // w_N^t = lo[t & (2^bits - 1)] * hi[t >> bits]
    int32_t itw_bits;
    int32_t pass;
    double tau_coef;    // tau = tau_coef * sqrt(S)
    DevReport *rep;
    DevRecord *recs;
    int64_t rec_cap;
    const int32_t *fault_head; // [n_groups] first fault of each group or -1; NULL if none
    const DevFault *faults;
    // element offset of each signal in the input / output buffer (ragged
    // batches); NULL: signal b starts at b * N
    const int64_t *in_sig, *out_sig;
    double kappa_u;     // FT_THREAD: kappa * unit roundoff (butterfly thresholds)
    int32_t fix;        // FT_THREAD: recompute a flagged butterfly (CORRECT mode)
    int32_t m1_log2;    // LAST: log2(m1), so that the row map shifts instead of dividing
    int64_t g_base;     // index of this launch's first group within the pass (a chunk of the
                        // batch): fault lookup and records use g_base + g
    int32_t task;       // persistent ragged kernel: task index carried by the records (0 otherwise)
    int32_t ns_log2;    // multi-pass: log2(n_strips)
    int32_t o_log2;     // STRIDED: log2(O)
    int32_t pad_;
};

// Checksum schemes of a pass kernel (template argument FT).
enum { FT_NONE = 0, FT_BLOCK = 1, FT_SIGNAL = 2, FT_THREAD = 3 };

// ------------------------------------------------ persistent ragged queue
// A task is one pass of one length class of a ragged batch; an item is a
// range of the task's checksum groups; a chunk is a block of the class's
// signals (a whole number of every pass's checksum groups) whose items of
// pass p must all be released before its items of pass p + 1 start.
struct PItem {
    int32_t task;
    int32_t chunk;
    int64_t g0, g1;  // groups g0, g0 + step, ... below g1 of the task's pass
    int64_t step;
};
struct PTask {
    PassArgs a;         // the pass: tables, buffers, geometry, report (g_base = 0)
    int32_t variant;    // compiled kernel variant, pvariant_id(kind, M)
    int32_t dep;        // task of the previous pass of the same class, -1 for none
    int32_t done_base;  // index of this task's chunk 0 in the done / need arrays
    int32_t fix;        // correct flagged groups before releasing the item
    int32_t publish;    // a later pass reads this task's output: release the items
    int32_t pad_;
};
struct PQueue {
    const PItem *items;        // the queues' items, queue after queue
    int64_t n_items;           // all queues together
    const PTask *tasks;
    unsigned long long *head;  // next item to take, per queue
    const int64_t *q_begin;    // queue k holds items [q_begin[k], q_begin[k + 1])
    int32_t n_queues;          // 1..kPQueues
    int32_t pad_;
    int32_t *done;             // items released, per (task, chunk)
    const int32_t *need;       // items, per (task, chunk)
    int32_t *err;              // bit 0: a dependency wait ran out; bit 1: unknown variant
    int64_t spin_limit;        // polls of a dependency wait before it gives up
};
constexpr int kPQueues = 8;  // at most one work queue per XCD
constexpr int pvariant_id(int kind, int M) { return kind * 16 + ilog2c(M); }
constexpr int kPersistThreads = 512;  // threads of the persistent workgroup
constexpr int kPSlotCap = 64;         // groups per item (each flags at most one record)

// Size of the library's static device scratch (one copy per device), the
// memory of the allocation-free entry point: report counters, records and
// multi-pass workspace of one execution.
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of the scratch on `device` (the current device); NULL on
// failure.
void *scratch_address(int device);

// Host-side launchers (defined in the kernel translation unit).
hipError_t launch_pass(int fp64, int M, int kind, int ft, const PassArgs &a, int grid, hipStream_t st);
hipError_t launch_correct(int fp64, int M, int kind, const PassArgs &a, int grid, hipStream_t st);
hipError_t launch_reset(DevReport *rep, hipStream_t st);
// Persistent ragged kernel: launch over `grid` workgroups, its resident
// workgroups per compute unit, and the reset of its queue state and report.
hipError_t launch_persist(int fp64, int ft, const PQueue &q, int grid, hipStream_t st);
int persist_occupancy(int fp64, int ft);
hipError_t launch_persist_reset(const PQueue &q, int n_done, DevReport *rep, hipStream_t st);
// Streaming device copy of `bytes` (measurement instrument).
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t st);
// Resident workgroups of a pass kernel per compute unit (0 on error).
int pass_occupancy(int fp64, int M, int kind, int ft);

}  // namespace tfft
