#pragma once
// Persistent ragged execution (device side): one kernel launch drains a
// queue of work items across the length classes of a ragged batch.  An item
// is a range of checksum groups of one pass of one class (a "task"); the
// workgroup that takes it runs the pass kernel's group loop on that range
// (pass_body, with tiles widened to fill 512 threads), corrects the groups of
// the range that it flagged (CORRECT mode, binary64, from the group's combined
// input: the delayed, batched correction of Section III-B, done before the
// data move on), and releases the item.  Items of pass p > 0 of a class wait
// until every item of pass p - 1 covering the same block of signals (a
// "chunk") is released.  The items sit in up to 8 queues (one per XCD), all
// items of a chunk in the same queue; a workgroup takes items from its own
// queue, then from the others once it is drained.  Each queue's items are
// taken in order and an item only waits on items earlier in its own queue,
// which running workgroups hold: the waits end whatever the number of
// resident workgroups.  Each wait is
// bounded all the same (an error flag, then the workgroup moves on), so every
// wavefront reaches the end of the kernel.
#include "tfft_kernels.h"

namespace tfft {

constexpr int kPThreads = kPersistThreads;

// The compiled variants: one-pass rows of 64..4096 points, strided and last
// passes of 64..1024 points.
#define TFFT_PVARIANTS(X)                                                                                   \
    X(KIND_ROWS, 64) X(KIND_ROWS, 128) X(KIND_ROWS, 256) X(KIND_ROWS, 512) X(KIND_ROWS, 1024)                \
    X(KIND_ROWS, 2048) X(KIND_ROWS, 4096) X(KIND_STRIDED, 64) X(KIND_STRIDED, 128) X(KIND_STRIDED, 256)      \
    X(KIND_STRIDED, 512) X(KIND_STRIDED, 1024) X(KIND_LAST, 64) X(KIND_LAST, 128) X(KIND_LAST, 256)          \
    X(KIND_LAST, 512) X(KIND_LAST, 1024)

template <typename R, int FT, int KIND, int M>
constexpr size_t pvariant_lds() {
    const size_t pass = sizeof(PassShared<R, M, KIND, FT, kPThreads>);
    const size_t corr = sizeof(cx<double>) * M;  // the correction's binary64 transform
    return pass > corr ? pass : corr;
}

template <typename R, int FT>
constexpr size_t persist_pool_bytes() {
    size_t m = 0;
#define TFFT_PV_MAX(K, MM) m = pvariant_lds<R, FT, K, MM>() > m ? pvariant_lds<R, FT, K, MM>() : m;
    TFFT_PVARIANTS(TFFT_PV_MAX)
#undef TFFT_PV_MAX
    return (m + 15) / 16 * 16;
}
// the LDS-DMA prefetch buffer, an LDS variable of its own (as in pass_kernel)
template <typename R, int FT>
constexpr size_t persist_nbuf_bytes() {
    size_t m = 0;
#define TFFT_PV_NB(K, MM)                                                         \
    m = sizeof(cx<R>) * pass_nbuf_elems<R, MM, K, FT, kPThreads>() > m            \
            ? sizeof(cx<R>) * pass_nbuf_elems<R, MM, K, FT, kPThreads>()          \
            : m;
    TFFT_PVARIANTS(TFFT_PV_NB)
#undef TFFT_PV_NB
    return (m + 15) / 16 * 16;
}

// Wait until *p >= target, then acquire at agent scope; false after `limit`
// polls.  The polls are relaxed atomic loads and the acquire is one fence
// after the last: an acquiring load per poll would invalidate the caches of
// the workgroup's chiplet at every poll, under the feet of the workgroups
// still streaming through them.
__device__ __forceinline__ bool wait_count(const int32_t *p, int32_t target, int64_t limit) {
    int64_t n = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++n > limit) return false;
        __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// The item and task tables are read-only for the whole launch and passed as
// restrict-qualified arguments, so that their uniform loads become scalar
// loads and a task's PassArgs stays in scalar registers.
template <typename R, int FT>
__global__ void __launch_bounds__(kPThreads) persist_kernel(PQueue q, const PItem *__restrict__ items,
                                                            const PTask *__restrict__ tasks) {
    constexpr size_t POOL = persist_pool_bytes<R, FT>();
    constexpr size_t NPOOL = persist_nbuf_bytes<R, FT>();
    static_assert(POOL + NPOOL <= 150 * 1024, "persistent kernel LDS");
    __shared__ __align__(16) unsigned char pool[POOL];
    __shared__ __align__(16) unsigned char npool[NPOOL];
    __shared__ int64_t slots[kPSlotCap];
    __shared__ int n_slots;
    __shared__ int64_t cur;
    __shared__ double scratch[kPThreads / 64];
    // Every branch of the item loop itself is wave-uniform: the queue and
    // release work is done by wavefront 0 as a whole (its lanes agree, and
    // only lane 0 contributes to an atomic sum), never under a lane test.  A
    // lane-divergent `if (tid == 0)` next to the loop's back edge lets the
    // compiler take that lane out of the loop while the others go round
    // again past the barrier, with the previous item's index.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    auto uniform64 = [](int64_t v) -> int64_t {
        const uint64_t u = (uint64_t)v;
        return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)u));
    };
    // Queues: workgroup b serves queue b mod n_queues first (consecutive
    // workgroups run on different XCDs, so each XCD works through the items
    // of its own queue), then the others in turn once its own is drained.
    // Every item's dependencies sit earlier in its own queue, and a queue's
    // items are taken in order, so the waits end as with a single queue.
    const int home = (int)(blockIdx.x % (unsigned)q.n_queues);
    int tried = 0;  // queues found drained (wavefront 0)
    for (;;) {
        if (wave == 0) {
            int64_t got = -1;
            while (__builtin_amdgcn_readfirstlane(tried) < q.n_queues) {
                const int k = __builtin_amdgcn_readfirstlane((home + tried) % q.n_queues);
                // one increment per workgroup: lane 0 adds 1, the others 0
                const int64_t t = uniform64((int64_t)atomicAdd(q.head + k, (unsigned long long)one));
                const int64_t b0 = q.q_begin[k], b1 = q.q_begin[k + 1];
                if (b0 + t < b1) {
                    got = b0 + t;
                    break;
                }
                ++tried;
            }
            cur = got;  // -1: every queue drained
        }
        __syncthreads();
        const int64_t it = uniform64(cur);
        if (it < 0) break;
        const PItem item = items[it];
        const PTask &tk = tasks[item.task];
        const int variant = __builtin_amdgcn_readfirstlane(tk.variant);
        const int dep = __builtin_amdgcn_readfirstlane(tk.dep);
        const int done_at = __builtin_amdgcn_readfirstlane(tk.done_base + item.chunk);
        const int fix = __builtin_amdgcn_readfirstlane(tk.fix);
        const int publish = __builtin_amdgcn_readfirstlane(tk.publish);
        const PassArgs &a = tk.a;
        if (wave == 0) {
            if (dep >= 0) {
                // the previous pass of these signals, released by its items
                const PTask &pt = tasks[dep];
                const int at = __builtin_amdgcn_readfirstlane(pt.done_base + item.chunk);
                if (!wait_count(q.done + at, q.need[at], q.spin_limit)) atomicOr(q.err, 1);
            }
            n_slots = 0;
        }
        __syncthreads();
        const PassHooks hk{slots, &n_slots, kPSlotCap};
        switch (variant) {
#define TFFT_PV_RUN(K, MM)                                                                                     \
    case pvariant_id(K, MM):                                                                                   \
        pass_body<R, MM, K, FT, kPThreads>(a, *reinterpret_cast<PassShared<R, MM, K, FT, kPThreads> *>(pool), \
                                           reinterpret_cast<cx<R> *>(npool), item.g0, item.g1, item.step, hk); \
        break;
            TFFT_PVARIANTS(TFFT_PV_RUN)
#undef TFFT_PV_RUN
            default:
                if (wave == 0) atomicOr(q.err, 2);
                break;
        }
        __syncthreads();
        if constexpr (FT == FT_BLOCK) {
            // the flagged groups of this item, corrected before it is released
            const int ns = __builtin_amdgcn_readfirstlane(n_slots);
            if (fix && ns > 0) {
                for (int k = 0; k < ns; ++k) {
                    const int64_t slot = uniform64(slots[k]);
                    if (slot >= a.rec_cap) continue;  // dropped record: reported as such
                    switch (variant) {
#define TFFT_PV_FIX(K, MM)                                                                               \
    case pvariant_id(K, MM):                                                                             \
        correct_record<R, MM, K, PassCfg<R, MM, K, FT, kPThreads>::C, kPThreads>(                        \
            a, slot, reinterpret_cast<cx<double> *>(pool), scratch);                                     \
        break;
                        TFFT_PVARIANTS(TFFT_PV_FIX)
#undef TFFT_PV_FIX
                        default:
                            break;
                    }
                }
            }
        }
        // release (when a later pass reads this output): every wavefront's
        // stores visible at agent scope, then the count
        if (publish) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (wave == 0 && publish)
            __hip_atomic_fetch_add(q.done + done_at, (int32_t)one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename R, int FT>
hipError_t persist_launch(const PQueue &q, int grid, hipStream_t st) {
    hipLaunchKernelGGL((persist_kernel<R, FT>), dim3(grid), dim3(kPThreads), 0, st, q, q.items, q.tasks);
    return hipGetLastError();
}

template <typename R, int FT>
int persist_occ() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_kernel<R, FT>, kPThreads, 0) != hipSuccess) return 0;
    return n;
}

#define TFFT_PERSIST_INSTANTIATE(R, FT)                                                \
    template hipError_t persist_launch<R, FT>(const PQueue &, int, hipStream_t); \
    template int persist_occ<R, FT>();
#define TFFT_PERSIST_EXTERN(R, FT)                                                            \
    extern template hipError_t persist_launch<R, FT>(const PQueue &, int, hipStream_t); \
    extern template int persist_occ<R, FT>();

}  // namespace tfft
