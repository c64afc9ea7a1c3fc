// Device side of the SMMO heap: hierarchical bitmaps, block slot reservation
// and release, block invalidation, and wavefront-aggregated allocation and
// deallocation.  Follows the DynaSOAr allocator (Springer, Ch.5 sec.5.2 and
// sec.5.3, correctness argument in sec.5.4), re-expressed for CDNA wave64:
//   - a block holds 64 objects, so its 64-bit allocation bitmap is exactly a
//     wavefront ballot; one wavefront processes one block, one lane per slot;
//   - the leader of an aggregated allocation is the lowest requesting lane,
//     results are broadcast by readlane and ranks come from the ballot;
//   - CDNA has no independent thread scheduling, so every retrying bitmap
//     update runs in a converged loop in which each lane tries each of its
//     pending updates once per iteration (the deadlock-free deallocation of
//     sec.5.4.4, applied to every multi-lane bitmap update);
//   - every retry loop is bounded; exceeding the bound raises a device error
//     instead of hanging the GPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smmo_layout.hpp"

namespace smmo {

// ---------------------------------------------------------------- atomics --
// Bitmap words and block headers are shared mutable state; all accesses go
// through agent-scope atomics, which are performed at the device's point of
// coherence (past the per-CU L1 and the per-XCD L2).  They are relaxed: an
// acquire or release at agent scope makes the compiler write back and
// invalidate the whole L2 of the XCD around the atomic, which on this chip
// costs far more than the atomic.  The orderings the allocator needs are
// among these atomics themselves: a thread's atomic whose result it uses has
// been performed before its next access is issued, and a block-type store is
// made complete (complete_prior) before the bitmap update that publishes
// it.  Object data written by methods is published at kernel boundaries.
__device__ __forceinline__ uint64_t ald(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ald32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t aor(uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t aand(uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// waits until every earlier memory access of this thread (stores included)
// has been performed
__device__ __forceinline__ void complete_prior() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void raise_error(const HeapView &h, uint32_t bits)
{
    __hip_atomic_fetch_or(h.ctrl + CTRL_ERR, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// adds n to event counter `ev` in this wavefront's stripe
__device__ __forceinline__ void count_events(const HeapView &h, uint32_t ev, uint64_t n)
{
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint32_t *w = h.ctrl + CTRL_EVENTS + (wave % kEventStripes) * kStripeWords + ev;
    __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(w), (unsigned long long)n,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void count_event(const HeapView &h, uint32_t ev) { count_events(h, ev, 1); }

// the block list of class cls (wave-uniform)
__device__ __forceinline__ BlockList block_list(const HeapView &h, uint32_t cls)
{
    BlockList L;
    L.R = h.R + (uint64_t)cls * h.M;
    L.M = h.M;
    L.direct = (h.direct >> cls) & 1;
    if (L.direct) {
        L.r = L.nd = h.M;
        return L;
    }
    L.r = __builtin_amdgcn_readfirstlane(__hip_atomic_load(h.ctrl + CTRL_RFINAL + cls, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t ns = __builtin_amdgcn_readfirstlane(__hip_atomic_load(h.ctrl + CTRL_RSFINAL + cls,
                                                                         __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT));
    L.nd = L.r - ns;
    return L;
}

__device__ __forceinline__ bool heap_failed(const HeapView &h)
{
    return ald32(h.ctrl + CTRL_ERR) != 0;
}

// ------------------------------------------------------------ bit helpers --
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// a value every lane holds alike, moved to scalar registers
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t rotr64(uint64_t x, uint32_t r)
{
    r &= 63;
    return r ? (x >> r) | (x << (64 - r)) : x;
}

// index of the n-th (0-based) set bit of b, or 64 if b has fewer bits
// (Alg. nth_set_bit: clear the lowest set bit n times, then find first set)
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t b, uint32_t n)
{
    for (uint32_t i = 0; i < n && b; ++i) b &= b - 1;
    return b ? (uint32_t)(__ffsll((unsigned long long)b) - 1) : 64u;
}

// the lowest n set bits of b
__device__ __forceinline__ uint64_t lowest_bits(uint64_t b, uint32_t n)
{
    if ((uint32_t)__popcll(b) <= n) return b;
    uint32_t p = nth_set_bit(b, n);   // first bit not taken
    return b & ((1ull << p) - 1);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__device__ __forceinline__ uint32_t global_wave_id()
{
    return blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
}

// ---------------------------------------------------- hierarchical bitmap --
// A bitmap of M bits is a stack of levels; level l+1 has one bit per 64-bit
// container of level l, set iff that container is non-zero ("container
// consistency", sec.5.3.1).  Levels are only eventually consistent while
// kernels run; they are consistent whenever no kernel runs on the heap.

// One pending switch of a bit: dir +1 = set (0 -> 1), -1 = clear (1 -> 0).
// A successful switch that sets the first bit of a container, or clears its
// last bit, continues as the same switch one level up (Alg. try_clear).
struct BitOp {
    uint32_t pos;
    uint16_t bmid;
    int8_t lvl;
    int8_t dir;
};

constexpr int kMaxOps = 6;

// Invalidation attempts of one block (Alg. invalidate with rollback) before
// the release that emptied it gives up, and the most switches one release
// queues: a re-activation, a rollback per failed attempt but the last, and
// the three switches of a successful invalidation.
constexpr int kInvalidateAttempts = kMaxOps - 3;
constexpr int kMaxReleaseOps = 1 + (kInvalidateAttempts - 1) + 3;
static_assert(kMaxReleaseOps <= kMaxOps, "a release can queue more bitmap switches than the queue holds");

// A lane's queue of pending switches.  A push into a full queue is not
// dropped silently: it marks the queue, and completing the queue raises
// ERR_INTERNAL (run_ops_wave, run_ops_lane).
struct OpQueue {
    BitOp op[kMaxOps];
    bool overflow;
    __host__ __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int i = 0; i < kMaxOps; ++i) op[i].dir = 0;
        overflow = false;
    }
    __host__ __device__ __forceinline__ bool push(uint32_t bmid, uint32_t pos, int dir)
    {
#pragma unroll
        for (int i = 0; i < kMaxOps; ++i)
            if (op[i].dir == 0) {
                op[i].pos = pos;
                op[i].bmid = (uint16_t)bmid;
                op[i].lvl = 0;
                op[i].dir = (int8_t)dir;
                return true;
            }
        overflow = true;
        return false;
    }
    __host__ __device__ __forceinline__ bool pending() const
    {
        bool p = false;
#pragma unroll
        for (int i = 0; i < kMaxOps; ++i) p |= op[i].dir != 0;
        return p;
    }
};

// One attempt of a pending switch.  A failed attempt (the bit already has the
// target value: another thread's opposite switch is still on its way) leaves
// the op pending; the caller retries it later.
__device__ __forceinline__ void bitop_try(const HeapView &h, BitOp &o)
{
    uint64_t *w = h.bm_word(o.bmid, (uint32_t)o.lvl, o.pos >> 6);
    const uint64_t bit = 1ull << (o.pos & 63);
    if (o.dir > 0) {
        const uint64_t prev = aor(w, bit);
        if (prev & bit) return;
        if (prev == 0 && (uint32_t)o.lvl + 1 < h.nlev) {
            o.lvl++;
            o.pos >>= 6;
            return;
        }
        o.dir = 0;
    } else {
        const uint64_t prev = aand(w, ~bit);
        if (!(prev & bit)) return;
        if (prev == bit && (uint32_t)o.lvl + 1 < h.nlev) {
            o.lvl++;
            o.pos >>= 6;
            return;
        }
        o.dir = 0;
    }
}

// Converged completion of every lane's pending switches.  All lanes of the
// wavefront that may hold pending switches must call this together; each
// iteration every lane tries each of its pending switches once, so a switch
// that waits for another lane's switch cannot block it.
__device__ __forceinline__ void run_ops_wave(const HeapView &h, OpQueue &q)
{
    if (q.overflow) raise_error(h, ERR_INTERNAL);
    for (uint32_t it = 0;; ++it) {
        bool pend = false;
#pragma unroll
        for (int i = 0; i < kMaxOps; ++i)
            if (q.op[i].dir) {
                bitop_try(h, q.op[i]);
                pend |= q.op[i].dir != 0;
            }
        const uint64_t pending = __ballot(pend);
        if (pending == 0) break;
        if (lane_id() == (uint32_t)(__ffsll((unsigned long long)pending) - 1)) count_event(h, EV_SPIN);
        if (it >= h.spin_limit) {
            if (pend) raise_error(h, ERR_SPIN);
            break;
        }
    }
}

// The same for a single lane running alone (the allocation leader: no other
// lane of its wavefront holds pending switches while it runs).
__device__ __forceinline__ void run_ops_lane(const HeapView &h, OpQueue &q)
{
    if (q.overflow) raise_error(h, ERR_INTERNAL);
    for (uint32_t it = 0; q.pending(); ++it) {
        if (it >= h.spin_limit) {
            raise_error(h, ERR_SPIN);
            return;
        }
        if (it) count_event(h, EV_SPIN);
#pragma unroll
        for (int i = 0; i < kMaxOps; ++i)
            if (q.op[i].dir) bitop_try(h, q.op[i]);
    }
}

__device__ __forceinline__ void switch_bit_lane(const HeapView &h, uint32_t bmid, uint32_t pos, int dir)
{
    OpQueue q;
    q.reset();
    q.push(bmid, pos, dir);
    run_ops_lane(h, q);
}

// Alg. try_find_set: top-down descent, at each level the first set bit of
// the container after rotating it by a seed-dependent amount ("Bitmap
// Rotation", sec.5.3.2).  May fail spuriously while levels are inconsistent.
__device__ __forceinline__ int64_t find_set(const HeapView &h, uint32_t bmid, uint32_t seed)
{
    count_event(h, EV_FIND);
    uint32_t idx = 0;
    for (int lvl = (int)h.nlev - 1; lvl >= 0; --lvl) {
        const uint64_t c = ald(h.bm_word(bmid, (uint32_t)lvl, idx));
        if (!c) return -1;
        const uint32_t r = h.rotation ? (hash32(seed + 0x9E3779B9u * (uint32_t)(lvl + 1)) & 63u) : 0u;
        const uint32_t b = ((uint32_t)(__ffsll((unsigned long long)rotr64(c, r)) - 1) + r) & 63u;
        idx = idx * 64u + b;
    }
    return (int64_t)idx;
}

// Bitmap::clear() on the free-block bitmap: find a set bit and switch it off;
// retry the search if another thread switched it first.  Returns -1 when no
// free block is found (the thesis spins forever here; we report exhaustion).
__device__ __forceinline__ int64_t claim_free_block(const HeapView &h, uint32_t seed)
{
    uint32_t misses = 0;
    for (uint32_t t = 0; t < h.spin_limit; ++t) {
        const int64_t b = find_set(h, BM_FREE, seed + t * 0x632BE5ABu);
        if (b < 0) {
            // A search can miss while another thread is between two levels
            // of the hierarchy; only a run of consecutive misses means the
            // heap is exhausted.  Races lost to other claimers (below) are
            // progress of others and do not count.
            if (++misses > 128u) return -1;
            __builtin_amdgcn_s_sleep(4);
            continue;
        }
        misses = 0;
        uint64_t *w = h.bm_word(BM_FREE, 0, (uint32_t)b >> 6);
        const uint64_t bit = 1ull << (b & 63);
        const uint64_t prev = aand(w, ~bit);
        if (!(prev & bit)) continue;           // someone else took it
        if (prev == bit && h.nlev > 1) {        // cleared the container's last bit
            OpQueue q;
            q.reset();
            q.op[0] = BitOp{(uint32_t)b >> 6, (uint16_t)BM_FREE, 1, -1};
            run_ops_lane(h, q);
        }
        return b;
    }
    raise_error(h, ERR_SPIN);
    return -1;
}

// Alg. initialize_block: publish the type, then reset the allocation bitmap
// (every class has capacity 64, so no tail bits are pre-set); both complete
// before the caller sets the block's allocated and active bits.
__device__ __forceinline__ void initialize_block(const HeapView &h, uint32_t bid, uint32_t cls)
{
    __hip_atomic_store(h.type + bid, cls, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    complete_prior();
    __hip_atomic_store(h.alloc_bm + bid, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    complete_prior();
}

// Block::reserve, extended to up to n slots at once (reserve_multiple):
// returns the mask of slots this call switched 0 -> 1 (0 = block full or
// invalidated) and whether this call made the block full.
__device__ __forceinline__ uint64_t reserve_slots(const HeapView &h, uint32_t bid, uint32_t n,
                                                  bool &filled)
{
    uint64_t *p = h.alloc_bm + bid;
    uint64_t cur = ald(p);
    filled = false;
    for (int it = 0; it < 64; ++it) {
        const uint64_t want = lowest_bits(~cur, n);
        if (!want) return 0;
        const uint64_t prev = aor(p, want);
        const uint64_t got = want & ~prev;
        if (got) {
            filled = (prev | want) == ~0ull;
            return got;
        }
        cur = prev | want;   // all wanted slots were taken meanwhile; look again
    }
    return 0;
}

// Alg. invalidate: try to switch all 64 slots to 1 so that no reservation can
// succeed; on success the block is empty and can be freed; if some slot was
// reserved meanwhile, roll back (and owe the deferred active-bit clear when a
// concurrent release saw the block as full).  Bitmap switches are queued,
// not performed, so that the caller can complete them in a converged loop.
// Returns true if the block was invalidated.
__device__ __forceinline__ bool invalidate_block(const HeapView &h, uint32_t bid, OpQueue &q)
{
    uint64_t *p = h.alloc_bm + bid;
    for (int attempt = 0; attempt < kInvalidateAttempts; ++attempt) {
        const uint64_t before = aor(p, ~0ull);
        if (before == ~0ull) return false;
        const uint32_t t = ald32(h.type + bid);
        if (before == 0) {
            // The block is ours and empty.  Retire its type before it is
            // marked free, so a stale block list sees it as not of class t
            // and a later initialize_block's store of a new type comes after.
            __hip_atomic_store(h.type + bid, kNull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            complete_prior();
            q.push(bm_active(t), bid, -1);
            q.push(bm_alloc(t), bid, -1);
            q.push(BM_FREE, bid, +1);
            return true;
        }
        const uint64_t before_rb = aand(p, before);
        if (before_rb != ~0ull) q.push(bm_active(t), bid, -1);
        if ((before_rb & before) != 0) return false;
        // empty again: retry the invalidation
    }
    return false;
}

// Block::deallocate for a set of slots of one block, with the block-state
// consequences of Alg. deallocate: the release that frees the first slot of a
// full block re-activates it; the release that empties it invalidates it.
// Switches are queued into q.
__device__ __forceinline__ void release_slots(const HeapView &h, uint32_t cls, uint32_t bid,
                                              uint64_t mask, OpQueue &q)
{
    const uint64_t prev = aand(h.alloc_bm + bid, ~mask);
    if ((prev & mask) != mask) {
        raise_error(h, ERR_BADHANDLE);   // releasing a free slot
        return;
    }
    count_events(h, EV_DELS, (uint64_t)__popcll(mask));
    if (prev == ~0ull) q.push(bm_active(cls), bid, +1);
    if ((prev & ~mask) == 0) invalidate_block(h, bid, q);
}

// ------------------------------------------------------------- allocation --
// The leader's part of Alg. allocate with request coalescing: find an active
// block of the class (lookup retry with rotation), else initialize a free
// block (slow path); reserve up to n slots; deactivate the block if this
// filled it; roll back if the block's type changed meanwhile.
__device__ __forceinline__ uint32_t leader_allocate(const HeapView &h, uint32_t cls, uint32_t n,
                                                    uint64_t &got, uint32_t seed, int64_t first = -1)
{
    got = 0;
    for (uint32_t attempt = 0; attempt < h.spin_limit; ++attempt) {
        // the first attempt may start from a block found in a prefetched
        // view of the active bitmap (wave_allocate with an ActiveView)
        int64_t bid = attempt == 0 ? first : -1;
        for (uint32_t t = 0; t < h.retries && bid < 0; ++t)
            bid = find_set(h, bm_active(cls), hash32(seed + attempt * 977u + t * 131u));
        if (bid < 0) {
            bid = claim_free_block(h, hash32(seed ^ (attempt * 0x27d4eb2fu)));
            if (bid < 0) {
                raise_error(h, ERR_NOMEM);
                return kNoBlock;
            }
            initialize_block(h, (uint32_t)bid, cls);
            switch_bit_lane(h, bm_alloc(cls), (uint32_t)bid, +1);
            switch_bit_lane(h, bm_active(cls), (uint32_t)bid, +1);
            count_event(h, EV_SLOW);
        }
        bool filled;
        const uint64_t g = reserve_slots(h, (uint32_t)bid, n, filled);
        if (g) {
            // issued after the reservation has been performed (its result
            // is used), so it sees the type published before the reset
            const uint32_t t = ald32(h.type + bid);
            if (filled) switch_bit_lane(h, bm_active(t), (uint32_t)bid, -1);
            if (t == cls) {
                got = g;
                count_events(h, EV_NEWS, (uint64_t)__popcll(g));
                return (uint32_t)bid;
            }
            OpQueue q;                     // block re-typed meanwhile: roll back
            q.reset();
            release_slots(h, t, (uint32_t)bid, g, q);
            run_ops_lane(h, q);
        }
        count_event(h, EV_RETRY);
    }
    raise_error(h, ERR_SPIN);
    return kNoBlock;
}

// A prefetched view of the upper part of class cls's active-block bitmap:
// lane i holds container i of level L = max(nlev - 2, 0), which has at most
// 64 containers (the level above it is one container).  Taken with plain
// loads before a method's allocation, in the same batch as the method's own
// loads, it lets the allocating wavefront skip the two top levels of the
// active-block search.  It is a hint: the reservation checks the block it
// picks, and a block that filled since the view was taken costs one retry
// through the ordinary search.
struct ActiveView {
    uint64_t w;
};

__device__ __forceinline__ ActiveView active_view(const HeapView &h, uint32_t cls)
{
    const uint32_t lvl = h.nlev >= 2 ? h.nlev - 2 : 0;
    const uint32_t lane = lane_id();
    ActiveView v;
    v.w = lane < h.lvl_n[lvl] ? *h.bm_word(bm_active(cls), lvl, lane) : 0ull;
    return v;
}

// The rest of Alg. try_find_set from a view: the container at level L and the
// bit in it picked as find_set picks them (the same rotations for the same
// seed), then the levels below L by loads.  Converged call; the result is
// wave-uniform (-1 if the view shows no active block).
__device__ __forceinline__ int64_t find_set_from_view(const HeapView &h, uint32_t bmid, const ActiveView &v,
                                                      uint32_t seed)
{
    const int lvl = h.nlev >= 2 ? (int)h.nlev - 2 : 0;
    const uint64_t nz = __ballot(v.w != 0);
    if (!nz) return -1;
    uint32_t idx = 0;
    if (h.nlev >= 2) {           // the single container above L, as the ballot
        const uint32_t r = h.rotation ? (hash32(seed + 0x9E3779B9u * (uint32_t)(lvl + 2)) & 63u) : 0u;
        idx = ((uint32_t)(__ffsll((unsigned long long)rotr64(nz, r)) - 1) + r) & 63u;
    }
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v.w, (int)idx);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v.w >> 32), (int)idx);
    uint64_t c = ((uint64_t)hi << 32) | lo;
    for (int l = lvl;; --l) {
        const uint32_t r = h.rotation ? (hash32(seed + 0x9E3779B9u * (uint32_t)(l + 1)) & 63u) : 0u;
        idx = idx * 64u + (((uint32_t)(__ffsll((unsigned long long)rotr64(c, r)) - 1) + r) & 63u);
        if (l == 0) break;
        c = uniform64(ald(h.bm_word(bmid, (uint32_t)l - 1, idx)));
        if (!c) return -1;
    }
    return (int64_t)idx;
}

// Allocation of one object of class `cls` for every lane with want = true.
// Must be called by all lanes of the wavefront together (converged).  With
// coalescing the lowest requesting lane allocates for all requesting lanes;
// each lane takes the slot whose rank among the reserved slots equals its
// rank among the requesting lanes.  Returns the handle, or SMMO_NULL when
// want is false or the heap is exhausted.
__device__ __forceinline__ uint32_t wave_allocate(const HeapView &h, uint32_t cls, bool want,
                                                  const ActiveView *view = nullptr)
{
    uint32_t result = kNull;
    uint64_t pending = __ballot(want);
    const uint32_t lane = lane_id();
    const uint32_t seed = hash32(global_wave_id() * 0x9E3779B1u + 0x51ED27u);
    for (uint32_t round = 0; pending; ++round) {
        const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)pending) - 1);
        const uint32_t n = h.coalescing ? (uint32_t)__popcll(pending) : 1u;
        uint32_t bid = kNoBlock;
        uint64_t got = 0;
        const uint32_t rseed = seed + round * 0x85ebca6bu;
        // the first round's first lookup from the view (seeded as the
        // ordinary search's first lookup would be)
        int64_t first = -1;
        if (view && round == 0) {
            if (lane == leader) count_event(h, EV_FIND);
            first = find_set_from_view(h, bm_active(cls), *view, hash32(rseed));
        }
        if (lane == leader) bid = leader_allocate(h, cls, n, got, rseed, first);
        bid = __shfl(bid, (int)leader);
        const uint32_t glo = __shfl((uint32_t)got, (int)leader);
        const uint32_t ghi = __shfl((uint32_t)(got >> 32), (int)leader);
        got = ((uint64_t)ghi << 32) | glo;
        if (bid == kNoBlock) break;
        const uint32_t k = (uint32_t)__popcll(got);
        if ((pending >> lane) & 1) {
            const uint32_t rank = (uint32_t)__popcll(pending & ((1ull << lane) - 1));
            if (rank < k) result = (bid << 6) | nth_set_bit(got, rank);
        }
        pending &= ~lowest_bits(pending, k);
    }
    return result;
}

// OR of v over the lanes of the wavefront (butterfly over both halves)
__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, d);
        hi |= (uint32_t)__shfl_xor((int)hi, d);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Deallocation of arbitrary handles of class `cls` (one per lane with want).
// Converged call.  Handles must name live objects of the class.  Lanes whose
// objects share a block are released together: one atomic per distinct
// block (the multi-slot release of sec.5.3.2), its bitmap switches completed
// before the next block's release.
__device__ __forceinline__ void wave_deallocate(const HeapView &h, uint32_t cls, uint32_t handle,
                                                bool want)
{
    const uint32_t lane = lane_id();
    uint64_t pending = __ballot(want);
    while (pending) {
        const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)pending) - 1);
        const uint32_t b = (uint32_t)__shfl((int)(handle >> 6), (int)leader);
        const bool mine = ((pending >> lane) & 1) && (handle >> 6) == b;
        const uint64_t slots = wave_or64(mine ? 1ull << (handle & 63) : 0ull);
        const uint64_t group = __ballot(mine);
        pending &= ~group;
        OpQueue q;
        q.reset();
        if (lane == leader) {
            // two lanes naming one object: released once, reported as a bad handle
            if (__popcll(slots) != __popcll(group)) raise_error(h, ERR_BADHANDLE);
            release_slots(h, cls, b, slots, q);
        }
        run_ops_wave(h, q);
    }
}

// Deallocation of objects that delete themselves inside a method: the
// wavefront processes one block, so all its releases go to that block and
// are combined into one atomic (the multi-slot release of sec.5.3.2).
// Converged call; `mask` is the ballot of the lanes deleting their object.
__device__ __forceinline__ void wave_release_own_block(const HeapView &h, uint32_t cls, uint32_t bid,
                                                       uint64_t mask)
{
    if (!mask) return;
    OpQueue q;
    q.reset();
    const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)mask) - 1);
    if (lane_id() == leader) release_slots(h, cls, bid, mask, q);
    run_ops_wave(h, q);
}

} // namespace smmo
