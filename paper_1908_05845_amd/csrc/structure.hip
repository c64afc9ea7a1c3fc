// structure (Ch.7 "structure"): a spring mesh with anchor, pull and free
// nodes that breaks under load; disconnected parts are found with a BFS and
// deleted (field contracts in include/smmo_methods.h).
//
// The node classes derive from an abstract NodeBase whose fields sit at the
// same offsets in every node class, so a spring reads either endpoint through
// one set of offsets whatever the endpoint's class, and a do-all on NodeBase
// is one launch per concrete node class (the library dispatches it).  The
// runtime type test of the thesis (cast<T>, from the object's address) is the
// block's type id here; since every launch covers one concrete class, the
// test on `this` is settled on the host at launch.
//
// Unlinking a spring decrements its endpoints' spring counts with an atomic,
// because several springs of one node may unlink in the same launch; the
// unlink that takes a count to zero deletes that node, which may belong to
// any node class: such deletions are grouped by block and released with the
// class read from the block's type id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

using namespace smmo;

namespace {

constexpr uint32_t kP2 = 0x80000000u;        // tag of a slot whose node is the spring's p2
constexpr int32_t kFar = SMMO_STRUCTURE_FAR;

struct StructK {
    uint32_t cls, spring_cls;
    // NodeBase fields (the same offsets in every node class)
    uint32_t n_x, n_y, n_spr, n_spr_stride, n_nspr, n_dist;
    // fields of the launched node class, where it has them
    uint32_t n_vx, n_vy, n_m;
    // Spring fields
    uint32_t s_p1, s_p2, s_k, s_L0, s_maxf, s_fx, s_fy, s_s1, s_s2, s_del;
    float dt;
    int32_t distance;
    uint32_t fam_mask;        // BFS methods: the concrete node classes one launch covers
    uint32_t anchor_mask;     // BFS methods: those of them that are AnchorNode or derive from it
    uint32_t *flag;
    uint32_t wpg;             // wavefronts per work-group of this launch (whole groups only)
};

constexpr uint32_t kMaxFamily = 4;   // concrete classes one family launch walks

// Calls f(bid, bm, cls), or f(bid, bm, cls, i), for every listed block of the
// classes in `mask` (at most kMaxFamily; wpg = the launch's wavefronts per
// work-group, passed in so that no load of the work-group size delays the
// walk), one wavefront per block: a grid-stride walk over their block lists
// taken one after the other, i = the block's position in that sequence.  Nothing is called once the heap
// has failed: the error word is read in the same batch of loads as the list
// lengths (the kernels that use this walker need no check of their own).  A listed block whose type changed
// comes with bm = 0 (no live slot), so f may load from any block it is given
// before it looks at bm (the loads then overlap the header's) but stores only
// to live slots.  The list lengths were written by earlier launches (the
// enumerations), so plain loads read them.
template <class F>
__device__ __forceinline__ void for_each_family_block(const HeapView &h, uint32_t mask, uint32_t wpg, F &&f)
{
    BlockList L[kMaxFamily];
    uint32_t cls[kMaxFamily], end[kMaxFamily], rf[kMaxFamily], rs[kMaxFamily];
    bool used[kMaxFamily];
    uint32_t total = 0, m = mask;
#pragma unroll
    for (uint32_t j = 0; j < kMaxFamily; ++j) {
        used[j] = m != 0;
        cls[j] = m ? (uint32_t)(__ffs(m) - 1) : 0u;
        m &= m - 1;
    }
    // the error word and all list lengths at once (an unused entry reads
    // class 0's words)
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
#pragma unroll
    for (uint32_t j = 0; j < kMaxFamily; ++j) {
        rf[j] = __builtin_amdgcn_readfirstlane(h.ctrl[CTRL_RFINAL + cls[j]]);
        rs[j] = __builtin_amdgcn_readfirstlane(h.ctrl[CTRL_RSFINAL + cls[j]]);
    }
    if (err) return;
#pragma unroll
    for (uint32_t j = 0; j < kMaxFamily; ++j) {
        L[j].R = h.R + (uint64_t)cls[j] * h.M;
        L[j].M = h.M;
        L[j].direct = (h.direct >> cls[j]) & 1;
        if (L[j].direct) {
            rf[j] = h.M;
            rs[j] = 0;
        }
        L[j].r = used[j] ? rf[j] : 0u;
        L[j].nd = used[j] ? rf[j] - rs[j] : 0u;
        total += L[j].r;
        end[j] = total;
    }
    const uint32_t nw = gridDim.x * wpg;
    for (uint32_t i = xcd_logical_wg() * wpg + (threadIdx.x >> 6); i < total; i += nw) {
        uint32_t bid = 0, c = 0;
#pragma unroll
        for (uint32_t j = 0; j < kMaxFamily; ++j) {
            const uint32_t start = end[j] - L[j].r;
            if (i >= start && i < end[j]) {       // exactly one segment holds entry i
                bid = L[j].at(i - start);
                c = cls[j];
            }
        }
        bid = __builtin_amdgcn_readfirstlane(bid);
        const uint32_t t = __builtin_amdgcn_readfirstlane(h.type[bid]);
        const uint64_t bm = uniform64(walk_bitmaps(h, c, false)[bid]);
        if constexpr (std::is_invocable_v<F &, uint32_t, uint64_t, uint32_t, uint32_t>)
            f(bid, t == c ? bm : 0ull, c, i);
        else
            f(bid, t == c ? bm : 0ull, c);
    }
}

__device__ __forceinline__ bool st_valid(const HeapView &h, uint32_t handle)
{
    if (handle != kNull && (handle >> 6) < h.M) return true;
    raise_error(h, ERR_BADHANDLE);
    return false;
}

// Deletes the objects named by `handle` on the lanes with want, of whatever
// class each block holds (the block's type id).  Converged call.  Lanes
// naming slots of one block are released together, one block per round.
__device__ __forceinline__ void wave_delete_any(const HeapView &h, uint32_t handle, bool want)
{
    const uint32_t lane = lane_id();
    uint64_t pending = __ballot(want);
    while (pending) {
        const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)pending) - 1);
        const uint32_t b = (uint32_t)__shfl((int)(handle >> 6), (int)leader);
        const bool mine = ((pending >> lane) & 1) && (handle >> 6) == b;
        const uint64_t slots = wave_or64(mine ? 1ull << (handle & 63) : 0ull);
        pending &= ~__ballot(mine);
        OpQueue q;
        q.reset();
        if (lane == leader) {
            const uint32_t cls = h.type[b];
            if (cls < h.nclasses) release_slots(h, cls, b, slots, q);
            else raise_error(h, ERR_BADHANDLE);
        }
        run_ops_wave(h, q);
    }
}

// Node::remove_spring for the spring in slot q of node `node`; returns true
// if it was the node's last spring (the caller deletes the node)
__device__ __forceinline__ bool unlink(const HeapView &h, const StructK &p, uint32_t node, uint32_t q)
{
    if (q >= 3) {
        raise_error(h, ERR_BADHANDLE);
        return false;
    }
    fref<uint32_t>(h, node, p.n_spr + q * p.n_spr_stride) = kNull;
    const int32_t prev = __hip_atomic_fetch_add(&fref<int32_t>(h, node, p.n_nspr), -1, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (prev <= 0) raise_error(h, ERR_INTERNAL);
    return prev == 1;
}

// a spring of this wavefront's block unlinks from both endpoints (want) and
// deletes itself, deleting the endpoints whose last spring it was
__device__ __forceinline__ void unlink_and_delete(const HeapView &h, const StructK &p, uint32_t bid, uint32_t s,
                                                  uint32_t a, uint32_t b, bool want)
{
    bool last_a = false, last_b = false;
    if (want) {
        last_a = unlink(h, p, a, farr<uint8_t>(h, bid, p.s_s1)[s]);
        last_b = unlink(h, p, b, farr<uint8_t>(h, bid, p.s_s2)[s]);
    }
    wave_delete_any(h, a, last_a);
    wave_delete_any(h, b, last_b);
    wave_release_own_block(h, p.spring_cls, bid, __ballot(want));
}

// AnchorPullNode::pull
__global__ __launch_bounds__(1024) void k_st_pull(HeapView h, StructK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        farr<float>(h, bid, p.n_x)[s] += farr<float>(h, bid, p.n_vx)[s] * p.dt;
        farr<float>(h, bid, p.n_y)[s] += farr<float>(h, bid, p.n_vy)[s] * p.dt;
    });
}

// Spring::force: tension-only Hooke's law; a spring pulled harder than its
// limit unlinks itself and is deleted.  The stretch and break decisions use
// one fixed float32 operation order (no contraction).  A wavefront works on
// U blocks at once: their fields are loaded before their headers are used,
// then all endpoint gathers are issued, then the forces computed.
template <int U>
__global__ __launch_bounds__(1024) void k_st_force(HeapView h, StructK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<U>(h, p.spring_cls, p.wpg, [&](const BlockHeads<U> &hd) {
#pragma clang fp contract(off)
        uint32_t a[U], b[U];
        float k[U], L0[U], maxf[U];
        // the blocks' own fields for all 64 slots (one contiguous run each)
#pragma unroll
        for (int j = 0; j < U; ++j) {
            a[j] = farr<uint32_t>(h, hd.bid[j], p.s_p1)[s];
            b[j] = farr<uint32_t>(h, hd.bid[j], p.s_p2)[s];
            k[j] = farr<float>(h, hd.bid[j], p.s_k)[s];
            L0[j] = farr<float>(h, hd.bid[j], p.s_L0)[s];
            maxf[j] = farr<float>(h, hd.bid[j], p.s_maxf)[s];
        }
        bool live[U];
        float xa[U], ya[U], xb[U], yb[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            live[j] = (hd.bm(j) >> s) & 1;
            if (live[j]) live[j] = st_valid(h, a[j]) && st_valid(h, b[j]);
            if (!live[j]) a[j] = b[j] = 0;
            xa[j] = ya[j] = xb[j] = yb[j] = 0.f;
            if (live[j]) {
                xa[j] = fref<float>(h, a[j], p.n_x);
                ya[j] = fref<float>(h, a[j], p.n_y);
                xb[j] = fref<float>(h, b[j], p.n_x);
                yb[j] = fref<float>(h, b[j], p.n_y);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!hd.own(j)) continue;   // (uniform over the wavefront)
            float fx = 0.f, fy = 0.f;
            bool brk = false;
            if (live[j]) {
                const float dx = xb[j] - xa[j];
                const float dy = yb[j] - ya[j];
                const float dy2 = dy * dy;
                const float l = __builtin_sqrtf(__builtin_fmaf(dx, dx, dy2));
                const float d = l - L0[j];
                const float F = k[j] * d;
                const bool stretched = l > L0[j];
                brk = stretched && F > maxf[j];
                if (stretched && !brk) {
                    const float c = k[j] * d / l;
                    fx = c * dx;
                    fy = c * dy;
                }
            }
            // full-width stores: dead, broken and slack slots get 0
            farr<float>(h, hd.bid[j], p.s_fx)[s] = fx;
            farr<float>(h, hd.bid[j], p.s_fy)[s] = fy;
            unlink_and_delete(h, p, hd.bid[j], s, a[j], b[j], brk);
        }
    });
}

// Node::update: the attached springs' forces in slot order, then v and x; U
// blocks at once, as in the force kernel
template <int U>
__global__ __launch_bounds__(1024) void k_st_node_update(HeapView h, StructK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<U>(h, p.cls, p.wpg, [&](const BlockHeads<U> &hd) {
        // the nodes' slots and own fields for all 64 slots (one contiguous run
        // each), before the gathers that depend on the slots
        uint32_t hs[U][3];
        float m[U], vx[U], vy[U], x[U], y[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
            for (int q = 0; q < 3; ++q) hs[j][q] = farr<uint32_t>(h, hd.bid[j], p.n_spr + q * p.n_spr_stride)[s];
            m[j] = farr<float>(h, hd.bid[j], p.n_m)[s];
            vx[j] = farr<float>(h, hd.bid[j], p.n_vx)[s];
            vy[j] = farr<float>(h, hd.bid[j], p.n_vy)[s];
            x[j] = farr<float>(h, hd.bid[j], p.n_x)[s];
            y[j] = farr<float>(h, hd.bid[j], p.n_y)[s];
        }
        // the gathers of all U blocks, live slots only
        float gx[U][3], gy[U][3];
        bool use[U][3];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool live = (hd.bm(j) >> s) & 1;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                gx[j][q] = gy[j][q] = 0.f;
                use[j][q] = false;
                if (!live || hs[j][q] == kNull) continue;
                const uint32_t sp = hs[j][q] & ~kP2;
                if (!st_valid(h, sp)) continue;
                use[j][q] = true;
                gx[j][q] = fref<float>(h, sp, p.s_fx);
                gy[j][q] = fref<float>(h, sp, p.s_fy);
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!((hd.bm(j) >> s) & 1)) continue;
            float Fx = 0.f, Fy = 0.f;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (!use[j][q]) continue;
                if (hs[j][q] & kP2) {
                    Fx -= gx[j][q];
                    Fy -= gy[j][q];
                } else {
                    Fx += gx[j][q];
                    Fy += gy[j][q];
                }
            }
            vx[j] += Fx / m[j] * p.dt;
            vy[j] += Fy / m[j] * p.dt;
            x[j] += vx[j] * p.dt;
            y[j] += vy[j] * p.dt;
            farr<float>(h, hd.bid[j], p.n_vx)[s] = vx[j];
            farr<float>(h, hd.bid[j], p.n_vy)[s] = vy[j];
            farr<float>(h, hd.bid[j], p.n_x)[s] = x[j];
            farr<float>(h, hd.bid[j], p.n_y)[s] = y[j];
        }
    });
}

// NodeBase::initialize_frontier (the cast to AnchorNode is the block's type)
__global__ __launch_bounds__(1024) void k_st_bfs_init(HeapView h, StructK p)
{
    for_each_family_block(h, p.fam_mask, p.wpg, [&](uint32_t bid, uint64_t bm, uint32_t t) {
        const uint32_t s = lane_id();
        if ((bm >> s) & 1) farr<int32_t>(h, bid, p.n_dist)[s] = ((p.anchor_mask >> t) & 1) ? 0 : kFar;
    });
}

// NodeBase::visit(distance).  Concurrent writers of a neighbour's distance
// all write distance + 1, and no node of this level's frontier changes.  The
// frontier flag is read only after the kernel, so plain stores of the same
// value suffice (the end of the kernel writes the caches back); a wavefront
// that already sees the flag set skips its store.  (Agent-scope stores to
// one word from every frontier wavefront would queue at that word.)
__global__ __launch_bounds__(1024) void k_st_bfs_visit(HeapView h, StructK p)
{
    for_each_family_block(h, p.fam_mask, p.wpg, [&](uint32_t bid, uint64_t bm, uint32_t) {
        const uint32_t s = lane_id();
        const int32_t dist = farr<int32_t>(h, bid, p.n_dist)[s];   // issued beside the header loads
        const bool front = (((bm >> s) & 1) != 0) & (dist == p.distance);   // no branch before the load
        const uint64_t fb = __ballot(front);
        if (fb && s == (uint32_t)(__ffsll((unsigned long long)fb) - 1) && *p.flag == 0) *p.flag = 1u;
        if (!front) return;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint32_t hs = farr<uint32_t>(h, bid, p.n_spr + q * p.n_spr_stride)[s];
            if (hs == kNull) continue;
            const uint32_t sp = hs & ~kP2;
            if (!st_valid(h, sp)) continue;
            const uint32_t o = fref<uint32_t>(h, sp, (hs & kP2) ? p.s_p1 : p.s_p2);
            if (!st_valid(h, o)) continue;
            int32_t &d = fref<int32_t>(h, o, p.n_dist);
            if (d == kFar) d = p.distance + 1;
        }
    });
}

// NodeBase::delete_node: an unvisited node flags its springs
__global__ __launch_bounds__(1024) void k_st_bfs_mark(HeapView h, StructK p)
{
    for_each_family_block(h, p.fam_mask, p.wpg, [&](uint32_t bid, uint64_t bm, uint32_t) {
        const uint32_t s = lane_id();
        const int32_t dist = farr<int32_t>(h, bid, p.n_dist)[s];
        if (!((((bm >> s) & 1) != 0) & (dist == kFar))) return;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint32_t hs = farr<uint32_t>(h, bid, p.n_spr + q * p.n_spr_stride)[s];
            if (hs != kNull && st_valid(h, hs & ~kP2)) fref<uint8_t>(h, hs & ~kP2, p.s_del) = 1;
        }
    });
}

// ---- BFS removal with a frontier queue ------------------------------------
// The same breadth-first search as the level-by-level visits above (every
// node's distance from the nearest anchor node, the nodes it never reaches
// deleted), with the frontier kept as a queue instead of found by a walk over
// every node block in every level.  During the search a node is named by a
// dense index, 64 i + slot for the block at position i of the node classes'
// block lists (taken one after the other), so that one visited bit per node
// slot fits the work-group's LDS for up to kBfsLdsBits slots.
// Workspace layout (uint32 words; cap = the node slots, 64 per block the node
// classes may hold; M = the heap's blocks):
//   [0, kBfsHeader)        header; word 0 = the number of anchor nodes
//   queue  [+cap)          the anchors' dense indices, then the frontier
//                          nodes that do not fit in LDS, level after level
//   rank   [+M)            per node block, its position in the lists
//   bits   [+cap / 32)     visited bits of the slots beyond the LDS bitmap
//                          (of all slots with SMMO_BFS_DEVICE_VISITED)
//   nbr    [+4 cap)        per dense index of a live node: its neighbours'
//                          dense indices (the other end of each spring slot,
//                          SMMO_NULL for an empty slot) and its handle
// The topology does not change during the search, so resolving each node's
// springs to its neighbours once, in one wide walk, takes two dependent loads
// out of every level's chain, and with the visited set in LDS a level's
// chain holds one load from device memory (the neighbour entry).
constexpr uint32_t kBfsHeader = 64;
constexpr uint32_t kBfsLdsQ = 2048;         // frontier nodes per LDS buffer (two buffers)
constexpr uint32_t kBfsLdsWords = 36800;    // the LDS visited bitmap: 1,177,600 slots
constexpr uint32_t kBfsLdsBits = 32 * kBfsLdsWords;
constexpr uint32_t kBfsThreads = 1024;      // the level kernel's one work-group

struct BfsLayout {
    uint64_t queue, rank, bits, nbr, words;
};

__host__ __device__ constexpr BfsLayout bfs_layout(uint64_t cap, uint64_t M)
{
    BfsLayout l{};
    l.queue = kBfsHeader;
    l.rank = l.queue + cap;
    l.bits = l.rank + M;
    l.nbr = (l.bits + cap / 32 + 3) & ~3ull;
    l.words = l.nbr + 4 * cap;
    return l;
}

__global__ __launch_bounds__(64) void k_st_bfs_clear(uint32_t *work)
{
    work[threadIdx.x] = 0u;
}

// the position of every node block in the lists, and its slots' visited
// bits in device memory cleared
__global__ __launch_bounds__(1024) void k_st_bfs_rank(HeapView h, StructK p, uint32_t *work, uint32_t cap)
{
    const BfsLayout L = bfs_layout(cap, h.M);
    for_each_family_block(h, p.fam_mask, p.wpg, [&](uint32_t bid, uint64_t, uint32_t, uint32_t i) {
        const uint32_t s = lane_id();
        if (64ull * i + 64 > cap) {
            if (s == 0) raise_error(h, ERR_INTERNAL);
            return;
        }
        if (s == 0) work[L.rank + bid] = i;
        if (s < 2) work[L.bits + 2 * i + s] = 0u;
    });
}

// NodeBase::initialize_frontier, appending the anchor nodes to the queue (one
// atomic per wavefront for all of its anchors), and each live node's
// neighbour entry
__global__ __launch_bounds__(1024) void k_st_bfs_queue_init(HeapView h, StructK p, uint32_t *work, uint32_t cap)
{
    const BfsLayout L = bfs_layout(cap, h.M);
    uint4 *nbr = reinterpret_cast<uint4 *>(work + L.nbr);
    const uint32_t *rank = work + L.rank;
    for_each_family_block(h, p.fam_mask, p.wpg, [&](uint32_t bid, uint64_t bm, uint32_t t, uint32_t i) {
        if (64ull * i + 64 > cap) return;   // (the rank pass has raised the error)
        const uint32_t s = lane_id();
        const uint32_t self = 64 * i + s;
        const bool live = ((bm >> s) & 1) != 0;
        const bool anchor = live && ((p.anchor_mask >> t) & 1);
        uint32_t hs[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) hs[q] = farr<uint32_t>(h, bid, p.n_spr + q * p.n_spr_stride)[s];
        if (live) {
            farr<int32_t>(h, bid, p.n_dist)[s] = anchor ? 0 : kFar;
            uint32_t other[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                other[q] = kNull;
                if (hs[q] == kNull || !st_valid(h, hs[q] & ~kP2)) continue;
                const uint32_t o = fref<uint32_t>(h, hs[q] & ~kP2, (hs[q] & kP2) ? p.s_p1 : p.s_p2);
                if (st_valid(h, o)) other[q] = o;
            }
            // a neighbour's dense index; one beyond the slots (a spring end
            // in a block the rank pass did not list) is an internal error,
            // not an index the search may use
            uint32_t o[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                o[q] = kNull;
                if (other[q] == kNull) continue;
                const uint64_t di = 64ull * rank[other[q] >> 6] + (other[q] & 63);
                if (di < cap) o[q] = (uint32_t)di;
                else raise_error(h, ERR_INTERNAL);
            }
            nbr[self] = make_uint4(o[0], o[1], o[2], (bid << 6) | s);
        }
        const uint64_t am = __ballot(anchor);
        if (!am) return;
        const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)am) - 1);
        uint32_t base = 0;
        if (s == leader) base = atomicAdd(work, (uint32_t)__popcll(am));
        base = (uint32_t)__shfl((int)base, (int)leader);
        const uint32_t pos = base + (uint32_t)__popcll(am & ((1ull << s) - 1));
        if (anchor) {
            if (pos < cap) work[L.queue + pos] = self;
            else raise_error(h, ERR_INTERNAL);
        }
    });
}

// NodeBase::visit for every level, in one work-group.  The visited set is a
// bitmap over dense indices, in LDS for the first kBfsLdsBits of them and in
// device memory beyond (or for all, SMMO_BFS_DEVICE_VISITED): a node is
// claimed by the atomic OR that sets its bit, so each node enters the
// frontier once, at its breadth-first distance.  Level d's frontier is an LDS
// part (up to qlim dense indices in one of two LDS buffers) followed by a
// range of the queue in device memory (level 0: the anchors; later: the
// appends that did not fit in LDS).  The threads share the frontier evenly:
// each writes a node's distance d, reads its neighbour entry and claims the
// neighbours; a node won is appended to level d + 1's frontier, at the
// position the LDS counter d mod 3 gives: below qlim in the other LDS
// buffer, beyond it in the queue after level d's own range.  One barrier
// ends a level, after which every thread knows the next frontier from that
// counter; the counter of level d + 1 was last read after the barrier that
// ended level d - 2, so thread 0 clears it during level d.  The loop ends at
// the first empty frontier, at most one level per node.  *levels = the
// number of levels the thesis's loop runs: the non-empty ones plus the pass
// that finds the frontier empty.
__global__ __launch_bounds__(kBfsThreads) void k_st_bfs_levels(HeapView h, StructK p, uint32_t *work, uint32_t cap,
                                                        uint32_t options, uint32_t *levels)
{
    __shared__ uint32_t s_bits[kBfsLdsWords];
    __shared__ uint32_t s_q[2][kBfsLdsQ];
    __shared__ uint32_t s_n0, s_stop, s_cnt[3];
    const BfsLayout L = bfs_layout(cap, h.M);
    uint32_t *queue = work + L.queue;
    uint32_t *gbits = work + L.bits;
    const uint4 *nbr = reinterpret_cast<const uint4 *>(work + L.nbr);
    const uint32_t lds_bits = (options & SMMO_BFS_DEVICE_VISITED) ? 0u : kBfsLdsBits;
    const uint32_t qlim = (options & SMMO_BFS_SMALL_FRONTIER) ? 64u : kBfsLdsQ;
    for (uint32_t w = threadIdx.x; w < kBfsLdsWords; w += kBfsThreads) s_bits[w] = 0u;
    if (threadIdx.x == 0) {
        s_stop = heap_failed(h) ? 1u : 0u;
        s_n0 = std::min(__hip_atomic_load(work, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), cap);
        s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
    }
    __syncthreads();
    if (s_stop) {
        if (threadIdx.x == 0) *levels = 0;
        return;
    }
    // sets the visited bit of dense index o; whether this call set it.
    // LdsOnly: every dense index is below lds_bits (a uniform choice, so the
    // level loop of a mesh that fits has no device-memory atomic at all)
    auto claim = [&](uint32_t o, auto lds_only) -> bool {
        const uint32_t bit = 1u << (o & 31);
        if (decltype(lds_only)::value || o < lds_bits) return (atomicOr(&s_bits[o >> 5], bit) & bit) == 0;
        return (atomicOr(&gbits[o >> 5], bit) & bit) == 0;
    };
    uint32_t nl = 0;                 // LDS part of the frontier, in s_q[cur]
    uint32_t glo = 0, ghi = s_n0;    // queue part of the frontier
    for (uint32_t i = threadIdx.x; i < ghi; i += kBfsThreads)
        if (!claim(queue[i], std::false_type{})) raise_error(h, ERR_INTERNAL);   // an anchor listed twice
    __syncthreads();
    uint32_t cur = 0;
    uint32_t d = 0;
    // one level: each node's three claims issued together (a missing
    // neighbour's claim is aimed at the node itself, visited already, so it
    // fails without a branch), then one append for all the node won, then
    // the node's distance (a store nothing in the level waits for)
    auto node = [&](uint32_t self, auto lds_only) {
        uint32_t *cnt = &s_cnt[d % 3];
        const uint4 e = nbr[self];
        const uint32_t o[3] = {e.x, e.y, e.z};
        bool won[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) won[q] = claim(o[q] == kNull ? self : o[q], lds_only);
        const uint32_t n = (uint32_t)won[0] + (uint32_t)won[1] + (uint32_t)won[2];
        // the wavefront's appends reserved by one LDS add: each lane's offset
        // is the sum of n over the active lanes below it, from ballots of n's
        // two bits (a per-lane add with a varying n would be turned into a
        // loop over the lanes)
        const uint64_t b0 = __ballot(n & 1), b1 = __ballot(n & 2);
        const uint64_t below = (1ull << lane_id()) - 1;
        const uint32_t tot = (uint32_t)(__popcll(b0) + 2 * __popcll(b1));
        uint32_t base = 0;
        if (tot) {   // (uniform over the active lanes)
            const uint32_t leader = (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1);
            if (lane_id() == leader) base = atomicAdd(cnt, tot);
            base = __builtin_amdgcn_readfirstlane(base);   // the leader is the first active lane
        }
        if (n) {
            uint32_t pos = base + (uint32_t)(__popcll(b0 & below) + 2 * __popcll(b1 & below));
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (!won[q]) continue;
                if (pos < qlim) {
                    s_q[cur ^ 1][pos] = o[q];
                } else {
                    const uint32_t g = ghi + (pos - qlim);
                    if (g < cap) queue[g] = o[q];
                    else raise_error(h, ERR_INTERNAL);
                }
                ++pos;
            }
        }
        fref<int32_t>(h, e.w, p.n_dist) = (int32_t)d;
    };
    // the frontier's LDS part and its queue part in separate branches, so
    // that each read is an LDS or a global load (not a flat one)
    auto level = [&](auto lds_only) {
        const uint32_t total = nl + (ghi - glo);
        for (uint32_t i = threadIdx.x; i < total; i += kBfsThreads) {
            if (i < nl) node(s_q[cur][i], lds_only);
            else node(queue[glo + (i - nl)], lds_only);
        }
    };
    const bool lds_only = cap <= lds_bits;
    for (;;) {
        if (nl + (ghi - glo) == 0) break;
        if (threadIdx.x == 0) s_cnt[(d + 1) % 3] = 0;
        if (lds_only) level(std::true_type{});
        else level(std::false_type{});
        __syncthreads();
        const uint32_t appended = s_cnt[d % 3];   // final: every append of the level precedes the barrier
        nl = std::min(appended, qlim);
        glo = ghi;
        ghi = std::min(ghi + (appended - nl), cap);
        cur ^= 1;
        ++d;
    }
    if (threadIdx.x == 0) *levels = d + 1;
}

// Spring::delete_spring
__global__ __launch_bounds__(1024) void k_st_bfs_delete(HeapView h, StructK p)
{
    for_each_block(h, p.spring_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        bool del = ((bm >> s) & 1) && farr<uint8_t>(h, bid, p.s_del)[s];
        uint32_t a = 0, b = 0;
        if (del) {
            a = farr<uint32_t>(h, bid, p.s_p1)[s];
            b = farr<uint32_t>(h, bid, p.s_p2)[s];
            del = st_valid(h, a) && st_valid(h, b);
        }
        unlink_and_delete(h, p, bid, s, a, b, del);
    });
}

// Spring::link: register the spring in its endpoints' slots
__global__ __launch_bounds__(1024) void k_st_link(HeapView h, StructK p)
{
    for_each_block(h, p.spring_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t a = farr<uint32_t>(h, bid, p.s_p1)[s], b = farr<uint32_t>(h, bid, p.s_p2)[s];
        const uint32_t q1 = farr<uint8_t>(h, bid, p.s_s1)[s], q2 = farr<uint8_t>(h, bid, p.s_s2)[s];
        if (!st_valid(h, a) || !st_valid(h, b)) return;
        if (q1 >= 3 || q2 >= 3) {
            raise_error(h, ERR_BADHANDLE);
            return;
        }
        const uint32_t me = (bid << 6) | s;
        fref<uint32_t>(h, a, p.n_spr + q1 * p.n_spr_stride) = me;
        fref<uint32_t>(h, b, p.n_spr + q2 * p.n_spr_stride) = me | kP2;
    });
}

enum Which { W_PULL, W_FORCE, W_NODE, W_BFS_INIT, W_BFS_VISIT, W_BFS_MARK, W_BFS_DELETE, W_LINK };

smmo_status bind_structure(smmo_heap *h, uint32_t cls, const smmo_structure_args &a, int which, StructK &k)
{
    const smmo_schema *sc = h->schema;
    const uint32_t nc = sc->nclasses;
    if (a.nodebase_class >= nc || a.anchor_class >= nc || a.spring_class >= nc)
        return fail(SMMO_EINVAL, "structure: class id out of range");
    const uint32_t nodes = class_family(sc, a.nodebase_class);
    if (!((nodes >> a.anchor_class) & 1) || ((nodes >> a.spring_class) & 1))
        return fail(SMMO_EINVAL, "structure: anchor class must derive from the node base, the spring class not");
    const bool on_spring = which == W_FORCE || which == W_BFS_DELETE || which == W_LINK;
    if (on_spring ? cls != a.spring_class : !((nodes >> cls) & 1))
        return fail(SMMO_EINVAL, "structure: method runs on a different class");
    memset(&k, 0, sizeof k);
    k.cls = cls;
    k.spring_cls = a.spring_class;
    const uint32_t nb = a.nodebase_class;
    BIND(nb, "x", SMMO_F32, 1, &k.n_x, nullptr);
    BIND(nb, "y", SMMO_F32, 1, &k.n_y, nullptr);
    BIND(nb, "springs", SMMO_HANDLE, 3, &k.n_spr, &k.n_spr_stride);
    BIND(nb, "nspr", SMMO_I32, 1, &k.n_nspr, nullptr);
    BIND(nb, "dist", SMMO_I32, 1, &k.n_dist, nullptr);
    if (which == W_PULL || which == W_NODE) {
        BIND(cls, "vx", SMMO_F32, 1, &k.n_vx, nullptr);
        BIND(cls, "vy", SMMO_F32, 1, &k.n_vy, nullptr);
    }
    if (which == W_NODE) BIND(cls, "m", SMMO_F32, 1, &k.n_m, nullptr);
    const uint32_t sp = a.spring_class;
    BIND(sp, "p1", SMMO_HANDLE, 1, &k.s_p1, nullptr);
    BIND(sp, "p2", SMMO_HANDLE, 1, &k.s_p2, nullptr);
    BIND(sp, "k", SMMO_F32, 1, &k.s_k, nullptr);
    BIND(sp, "L0", SMMO_F32, 1, &k.s_L0, nullptr);
    BIND(sp, "maxf", SMMO_F32, 1, &k.s_maxf, nullptr);
    BIND(sp, "fx", SMMO_F32, 1, &k.s_fx, nullptr);
    BIND(sp, "fy", SMMO_F32, 1, &k.s_fy, nullptr);
    BIND(sp, "s1", SMMO_U8, 1, &k.s_s1, nullptr);
    BIND(sp, "s2", SMMO_U8, 1, &k.s_s2, nullptr);
    BIND(sp, "del", SMMO_U8, 1, &k.s_del, nullptr);
    // the node fields every class of the family shares (same offsets)
    for (uint32_t c = 0; c < nc; ++c) {
        if (!((nodes >> c) & 1)) continue;
        uint32_t off = 0, stride = 0;
        const char *names[5] = {"x", "y", "springs", "nspr", "dist"};
        const uint32_t want[5] = {k.n_x, k.n_y, k.n_spr, k.n_nspr, k.n_dist};
        for (int f = 0; f < 5; ++f) {
            smmo_status s = bind_field(sc, c, names[f], f == 2 ? SMMO_HANDLE : (f < 2 ? SMMO_F32 : SMMO_I32),
                                       f == 2 ? 3 : 1, &off, f == 2 ? &stride : nullptr);
            if (s) return s;
            if (off != want[f]) return fail(SMMO_EINVAL, "structure: node classes disagree on a NodeBase field");
        }
    }
    // BFS methods: the concrete classes of the launched class's family
    const uint32_t fam = class_family(sc, cls), anchors = class_family(sc, a.anchor_class);
    for (uint32_t c = 0; c < nc; ++c)
        if (((fam >> c) & 1) && !class_abstract(sc, c)) k.fam_mask |= 1u << c;
    k.anchor_mask = k.fam_mask & anchors;
    if (__builtin_popcount(k.fam_mask) > (int)kMaxFamily)
        return fail(SMMO_EINVAL, "structure: more than 4 concrete node classes in one do-all");
    return SMMO_OK;
}

// the launch shape of a family launch: the method's shape, with as many
// wavefronts as the family's classes may have blocks
LaunchShape family_shape(smmo_heap *h, uint32_t cls, uint32_t mask)
{
    LaunchShape ls = method_shape(h, cls);
    uint64_t blocks = 0;
    for (uint32_t c = 0; c < h->schema->nclasses; ++c)
        if ((mask >> c) & 1) blocks += h->ub_blocks[c];
    // the family walks are latency-bound scans: a grid that is resident all at
    // once (32 wavefronts per CU) walks a BFS level faster than one twice as
    // large
    uint64_t waves = h->cfg.grid_waves ? h->cfg.grid_waves : 32ull * h->cu_count;
    if (h->cur_method < 64 && h->launch_waves[h->cur_method][cls]) waves = h->launch_waves[h->cur_method][cls];
    waves = std::min<uint64_t>(waves, std::max<uint64_t>(1, blocks));
    const uint32_t wpg = ls.block.x / 64;
    ls.grid = dim3((uint32_t)((waves + wpg - 1) / wpg));
    return ls;
}

template <int W>
smmo_status launch_structure(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_structure_args a;
    memcpy(&a, args, sizeof a);
    if (W == W_BFS_VISIT && !a.flag) return fail(SMMO_EINVAL, "structure.bfs_visit: flag is NULL");
    if (!(a.dt == a.dt)) return fail(SMMO_EINVAL, "structure: NaN dt");
    // the per-call fields do not take part in the binding
    smmo_structure_args key = a;
    key.distance = 0;
    key.dt = 0.f;
    key.bfs_options = 0;
    key.flag = nullptr;
    StructK k;
    smmo_status s = cached_bind(h, (const void *)&launch_structure<W>, cls, key, k,
                                [&] { return bind_structure(h, cls, a, W, k); });
    if (s) return s;
    k.dt = a.dt;
    k.distance = a.distance;
    k.flag = a.flag;
    const bool family = W == W_BFS_INIT || W == W_BFS_VISIT || W == W_BFS_MARK;
    LaunchShape ls;
    if (family) {
        for (uint32_t c = 0; c < h->schema->nclasses; ++c)
            if (((k.fam_mask >> c) & 1) && (s = ensure_enumerated(h, c, false, st))) return s;
        ls = family_shape(h, cls, k.fam_mask);
        if (!k.fam_mask) return SMMO_OK;
        k.wpg = ls.block.x / 64;
    } else {
        if ((s = ensure_enumerated(h, cls, false, st))) return s;
        // the force and node passes take blocks in groups (default one)
        ls = method_shape(h, cls, W == W_FORCE || W == W_NODE ? 1u : 0u);
        k.wpg = ls.block.x / 64;
    }
    switch (W) {
    case W_PULL: hipLaunchKernelGGL(k_st_pull, ls.grid, ls.block, 0, st, h->v, k); break;
    case W_FORCE:
        // a group of four blocks takes two at a time here: four need more
        // registers than a work-group of 1,024 threads leaves (it spills)
        if (ls.group >= 2) hipLaunchKernelGGL(k_st_force<2>, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_st_force<1>, ls.grid, ls.block, 0, st, h->v, k);
        break;
    case W_NODE:
        if (ls.group == 4) hipLaunchKernelGGL(k_st_node_update<4>, ls.grid, ls.block, 0, st, h->v, k);
        else if (ls.group == 2) hipLaunchKernelGGL(k_st_node_update<2>, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_st_node_update<1>, ls.grid, ls.block, 0, st, h->v, k);
        break;
    case W_BFS_INIT: hipLaunchKernelGGL(k_st_bfs_init, ls.grid, ls.block, 0, st, h->v, k); break;
    case W_BFS_VISIT: hipLaunchKernelGGL(k_st_bfs_visit, ls.grid, ls.block, 0, st, h->v, k); break;
    case W_BFS_MARK: hipLaunchKernelGGL(k_st_bfs_mark, ls.grid, ls.block, 0, st, h->v, k); break;
    case W_BFS_DELETE: hipLaunchKernelGGL(k_st_bfs_delete, ls.grid, ls.block, 0, st, h->v, k); break;
    default: hipLaunchKernelGGL(k_st_link, ls.grid, ls.block, 0, st, h->v, k); break;
    }
    return launched("structure kernel");
}

// BFS removal with the queue in `work` (words >= kBfsHeader + one per node
// slot of the family): queue set-up, all levels, then the mark and delete
// do-alls of the level-by-level form.
smmo_status remove_disconnected(smmo_heap *h, const smmo_structure_args &a, uint32_t *work, uint64_t words,
                                uint32_t *levels, hipStream_t st)
{
    smmo_status s = heap_check_class(h, a.nodebase_class);
    if (s) return s;
    if ((s = heap_check_class(h, a.spring_class))) return s;
    if (!work || !levels) return fail(SMMO_EINVAL, "structure BFS: workspace or level count is NULL");
    smmo_structure_args key = a;
    key.distance = 0;
    key.dt = 0.f;
    key.bfs_options = 0;
    key.flag = nullptr;
    StructK k;
    s = cached_bind(h, (const void *)&k_st_bfs_levels, a.nodebase_class, key, k,
                    [&] { return bind_structure(h, a.nodebase_class, key, W_BFS_INIT, k); });
    if (s) return s;
    if (a.bfs_options & ~(SMMO_BFS_DEVICE_VISITED | SMMO_BFS_SMALL_FRONTIER))
        return fail(SMMO_EINVAL, "structure BFS: unknown bfs_options bits");
    uint64_t slots = 0;
    for (uint32_t c = 0; c < h->schema->nclasses; ++c)
        if ((k.fam_mask >> c) & 1) slots += 64 * h->ub_blocks[c];
    if (slots > 0xFFFFFFFFull - kBfsHeader) return fail(SMMO_EINVAL, "structure BFS: too many node slots");
    if (words < bfs_layout(slots, h->v.M).words)
        return fail(SMMO_EINVAL, "structure BFS: the workspace needs 64 header words, 5 + 1/32 words per node slot "
                                 "of the node classes (64 per block they may hold), one word per block of the "
                                 "heap, and up to 3 words of alignment");
    // the dense indices are positions in the lists: enumerated lists, never
    // a direct walk over all blocks
    for (uint32_t c = 0; c < h->schema->nclasses; ++c)
        if (((k.fam_mask >> c) & 1) && (s = ensure_enumerated(h, c, false, st, false, false))) return s;
    const uint32_t cap = (uint32_t)slots;
    hipLaunchKernelGGL(k_st_bfs_clear, dim3(1), dim3(kBfsHeader), 0, st, work);
    if (k.fam_mask) {
        LaunchShape ls = family_shape(h, a.nodebase_class, k.fam_mask);
        k.wpg = ls.block.x / 64;
        hipLaunchKernelGGL(k_st_bfs_rank, ls.grid, ls.block, 0, st, h->v, k, work, cap);
        hipLaunchKernelGGL(k_st_bfs_queue_init, ls.grid, ls.block, 0, st, h->v, k, work, cap);
    }
    hipLaunchKernelGGL(k_st_bfs_levels, dim3(1), dim3(kBfsThreads), 0, st, h->v, k, work, cap, a.bfs_options, levels);
    if ((s = launched("structure BFS kernel"))) return s;
    h->last = st;
    if ((s = launch_structure<W_BFS_MARK>(h, a.nodebase_class, &a, st))) return s;
    return launch_structure<W_BFS_DELETE>(h, a.spring_class, &a, st);
}

} // namespace

smmo_status smmo_structure_remove_disconnected(smmo_heap *h, const smmo_structure_args *args, uint32_t *work,
                                               uint64_t work_words, uint32_t *levels, smmo_stream stream)
{
    if (!args) return fail(SMMO_EINVAL, "structure BFS: args is NULL");
    return remove_disconnected(h, *args, work, work_words, levels, static_cast<hipStream_t>(stream));
}

// ---- the same BFS without a caller workspace ------------------------------
// The workspace (queue, block positions, visited bits and neighbour table)
// lives in `scratch`, a device array of this library: each GPU the library
// runs on holds one copy, 21 MB, until the process ends.  It serves heaps of
// up to kScratchBlocks blocks.  In host code the array's name is not a
// device address; its address on a device is taken once per device
// (hipGetSymbolAddress, with that device current) and kept in scratch_ptr,
// which is what the kernels are given.  All calls on one GPU share the array
// and it keeps the last call's contents: the queue's header is cleared by a
// kernel at the start of every call (the rest is written before it is read),
// and calls that overlap on one GPU race.
constexpr uint32_t kScratchBlocks = 16384;
constexpr uint64_t kScratchWords = bfs_layout(64ull * kScratchBlocks, kScratchBlocks).words;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {
constexpr int kScratchDevices = 64;
uint32_t *scratch_ptr[kScratchDevices];
std::mutex scratch_mu;

smmo_status scratch_on(int device, uint32_t **out)
{
    if (device < 0 || device >= kScratchDevices) return fail(SMMO_EINVAL, "structure BFS: device id out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        scratch_ptr[device] = static_cast<uint32_t *>(p);
    }
    *out = scratch_ptr[device];
    return SMMO_OK;
}
} // namespace

smmo_status smmo_structure_remove_disconnected_noalloc(smmo_heap *h, const smmo_structure_args *args,
                                                       uint32_t *levels, smmo_stream stream)
{
    if (!h || !args) return fail(SMMO_EINVAL, "structure BFS: heap or args is NULL");
    int cur = -1;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != h->device) return fail(SMMO_EINVAL, "structure BFS: the heap's device must be the current device");
    if (h->v.M > kScratchBlocks)
        return fail(SMMO_EINVAL, "structure BFS without a workspace: the heap has more than 16,384 blocks (what "
                                 "the library's own array serves); pass a workspace instead");
    uint32_t *q = nullptr;
    smmo_status s = scratch_on(cur, &q);
    if (s) return s;
    return remove_disconnected(h, *args, q, kScratchWords, levels, static_cast<hipStream_t>(stream));
}

namespace smmo {
smmo_status launch_structure_pull(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_PULL>(h, c, a, s); }
smmo_status launch_structure_force(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_FORCE>(h, c, a, s); }
smmo_status launch_structure_node_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_NODE>(h, c, a, s); }
smmo_status launch_structure_bfs_init(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_BFS_INIT>(h, c, a, s); }
smmo_status launch_structure_bfs_visit(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_BFS_VISIT>(h, c, a, s); }
smmo_status launch_structure_bfs_mark(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_BFS_MARK>(h, c, a, s); }
smmo_status launch_structure_bfs_delete(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_BFS_DELETE>(h, c, a, s); }
smmo_status launch_structure_link(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_structure<W_LINK>(h, c, a, s); }
} // namespace smmo
