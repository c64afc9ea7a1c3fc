// Helpers shared by the method kernels (methods.hip, adjoint.hip): the
// block walk of a do-all, field access, and the per-heap cache of resolved
// field bindings.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/smmo_methods.h"
#include "smmo_device.hpp"
#include "smmo_host.hpp"

namespace smmo {

// Work-group g runs on XCD g % 8; give XCD x the contiguous range of logical
// work-group numbers [start(x), start(x) + count(x)).
__device__ __forceinline__ uint32_t xcd_logical_wg()
{
    const uint32_t G = gridDim.x, g = blockIdx.x;
    const uint32_t x = g & 7u, k = g >> 3, per = G >> 3, rem = G & 7u;
    return x * per + (x < rem ? x : rem) + k;
}


// The bitmaps a walk over class cls reads: the iteration bitmaps where the
// walk asks for the snapshot or the launch uses one that smmo_snapshot took
// before it (HeapView::snap), else the allocation bitmaps.
__device__ __forceinline__ const uint64_t *walk_bitmaps(const HeapView &h, uint32_t cls, bool snapshot)
{
    return snapshot || ((h.snap >> cls) & 1) ? h.iter_bm : h.alloc_bm;
}

// Calls f(bid, bitmap) for every block of class `cls` in R, one wavefront per
// block; nothing once the heap has failed (the error word is read in the
// same batch of loads as the list lengths).  A block that was freed (or freed and re-used by another class)
// since R was built has a different type and is skipped, so R may be a
// superset of the class's blocks.  bitmap = the iteration bitmap (snapshot of
// the allocation bitmap taken by the enumeration) or the allocation bitmap,
// as walk_bitmaps picks; the two are the same as long as nothing creates
// objects of the class after the snapshot.
// Within one launch a block's type and (outside snapshot mode) its bitmap
// change only through the wavefront that processes it, so plain loads are
// enough.  The next R entry is fetched one iteration ahead.
template <class F>
__device__ __forceinline__ void for_each_block(const HeapView &h, uint32_t cls, bool snapshot, F &&f)
{
    // the error word in the same batch of loads as the list lengths: nothing
    // is called once the heap has failed
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
    const BlockList L = block_list(h, cls);
    if (__builtin_amdgcn_readfirstlane(err)) return;
    const uint32_t r = L.r;
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t nw = gridDim.x * wpg;
    uint32_t i = xcd_logical_wg() * wpg + (threadIdx.x >> 6);
    if (i >= r) return;
    uint32_t bid = __builtin_amdgcn_readfirstlane(L.at(i));
    for (;;) {
        const uint32_t in = i + nw;
        const uint32_t bnext = __builtin_amdgcn_readfirstlane(in < r ? L.at(in) : 0u);
        const uint32_t t = __builtin_amdgcn_readfirstlane(h.type[bid]);
        const uint64_t bm = uniform64(walk_bitmaps(h, cls, snapshot)[bid]);
        if (t == cls) f(bid, bm);
        if (in >= r) break;
        i = in;
        bid = bnext;
    }
}

// The headers of the U blocks a wavefront takes in one iteration of
// for_each_block_heads: their ids, types and allocation bitmaps as loaded,
// and whether each R entry exists.  bm(j) is block j's bitmap if it is a
// block of the class, else 0.  Loading the headers and using them are
// separate steps, so a method can issue its loads from the blocks (which
// need only the ids) before it waits for the headers.
template <int U>
struct BlockHeads {
    uint32_t bid[U], type[U], cls;
    uint64_t raw[U];
    bool valid[U];
    __device__ __forceinline__ bool own(int j) const { return valid[j] && type[j] == cls; }
    __device__ __forceinline__ uint64_t bm(int j) const { return own(j) ? raw[j] : 0ull; }
};

// Calls f(heads) for the blocks of class `cls` in R, U at a time, as
// for_each_block_group walks them, with three differences that shorten the
// chain of dependent loads at the start of every wavefront: the error word
// is read in the same batch of loads as the list lengths (nothing is called
// once the heap has failed; a kernel using this walker needs no check of its
// own), the wavefronts per work-group are passed in (wpg) instead of read
// from the dispatch packet, and the block headers come to f unused.
// for_each_block_heads_in walks with work-group g of G (a part of the grid
// that starts at a multiple of eight work-groups, so that g mod 8 is still
// the work-group's XCD), so that one launch can walk two classes.
template <int U, class F>
__device__ __forceinline__ void for_each_block_heads_in(const HeapView &h, uint32_t cls, uint32_t wpg, uint32_t g,
                                                        uint32_t G, F &&f)
{
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
    const BlockList L = block_list(h, cls);
    if (__builtin_amdgcn_readfirstlane(err)) return;
    const uint32_t r = L.r;
    const uint32_t x = g & 7u;
    const uint32_t ngroups = (r + U - 1) / U;
    uint32_t glo = 0, ghi = ngroups, lw = g * wpg + (threadIdx.x >> 6), lstep = G * wpg;
    if (G >= 8) {
        glo = (uint32_t)((uint64_t)ngroups * x / 8);
        ghi = (uint32_t)((uint64_t)ngroups * (x + 1) / 8);
        lw = (g >> 3) * wpg + (threadIdx.x >> 6);
        lstep = ((G - x + 7) / 8) * wpg;
    }
    for (uint32_t gi = glo + lw; gi < ghi; gi += lstep) {
        const uint32_t base = gi * U;
        BlockHeads<U> hd;
        hd.cls = cls;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            hd.valid[j] = base + j < r;
            hd.bid[j] = __builtin_amdgcn_readfirstlane(L.at(hd.valid[j] ? base + j : base));
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            hd.type[j] = __builtin_amdgcn_readfirstlane(h.type[hd.bid[j]]);
            hd.raw[j] = uniform64(walk_bitmaps(h, cls, false)[hd.bid[j]]);
        }
        f(hd);
    }
}

template <int U, class F>
__device__ __forceinline__ void for_each_block_heads(const HeapView &h, uint32_t cls, uint32_t wpg, F &&f)
{
    for_each_block_heads_in<U>(h, cls, wpg, blockIdx.x, gridDim.x, f);
}

// Calls f(bid, bm, own) for the blocks of class `cls` in R, U at a time: a
// wavefront takes U consecutive R entries per iteration (consecutive blocks of
// an ordered bulk allocation, whose objects share their neighbours) and loads
// every block id, type and bitmap before f runs, so that f can issue the
// loads of all U blocks before it waits for any.  own[j] says whether entry j
// is a block of the class; for an entry past the end of R, bid[j] repeats a
// valid block and own[j] is false; bm[j] is 0 whenever own[j] is false.  f may
// load from any bid[j] but must store only to blocks it owns.
// R is split into eight contiguous ranges, one per XCD (work-group g runs on
// XCD g mod 8), walked by that XCD's wavefronts in grid-stride order; so a
// class's blocks and the blocks of another class that they gather from (in
// creation order: nodes and their springs) meet in the same L2 from one
// do-all to the next.  With fewer than eight work-groups the whole R is one
// range.
template <int U, class F>
__device__ __forceinline__ void for_each_block_group(const HeapView &h, uint32_t cls, F &&f)
{
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
    const BlockList L = block_list(h, cls);
    if (__builtin_amdgcn_readfirstlane(err)) return;
    const uint32_t r = L.r;
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t G = gridDim.x, g = blockIdx.x, x = g & 7u;
    const uint32_t ngroups = (r + U - 1) / U;
    uint32_t glo = 0, ghi = ngroups, lw = g * wpg + (threadIdx.x >> 6), lstep = G * wpg;
    if (G >= 8) {
        glo = (uint32_t)((uint64_t)ngroups * x / 8);
        ghi = (uint32_t)((uint64_t)ngroups * (x + 1) / 8);
        lw = (g >> 3) * wpg + (threadIdx.x >> 6);
        lstep = ((G - x + 7) / 8) * wpg;
    }
    for (uint32_t gi = glo + lw; gi < ghi; gi += lstep) {
        const uint32_t base = gi * U;
        uint32_t bid[U];
        uint64_t bm[U];
        bool own[U];
#pragma unroll
        for (int j = 0; j < U; ++j) bid[j] = __builtin_amdgcn_readfirstlane(L.at(base + j < r ? base + j : base));
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t t = __builtin_amdgcn_readfirstlane(h.type[bid[j]]);
            const uint64_t b = uniform64(walk_bitmaps(h, cls, false)[bid[j]]);
            own[j] = base + j < r && t == cls;
            bm[j] = own[j] ? b : 0;
        }
        f(bid, bm, own);
    }
}

// Calls f(bid, slot, live, pair) once per lane for the live objects of class cls
// (a packed do-all): a wavefront takes one dense block of the class's list
// (lane = slot), or two sparse blocks, lanes 0..31 serving the live slots of
// the first in slot order and lanes 32..63 those of the second.  bid and slot
// may differ between lanes; live is false for idle lanes (bid is then a valid
// block and slot 0); pair (wave-uniform) says whether the wavefront holds two
// blocks.  A block is never split across wavefronts, so the
// deletions of one block's objects by one launch are released together.  As
// in for_each_block, a listed block whose type is no longer cls is skipped.
// Packing halves the wavefronts the sparse blocks need; while the list is no
// longer than the grid every block already has a wavefront of its own, and
// packing would only lengthen the wavefronts that get two (sparse_packing 1
// then gives every block one wavefront; 0 never packs).  A list built without
// the packing plan lists every block as dense.
template <class F>
__device__ __forceinline__ void for_each_object_packed(const HeapView &h, uint32_t cls, bool snapshot, F &&f)
{
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
    const BlockList L = block_list(h, cls);
    if (__builtin_amdgcn_readfirstlane(err)) return;
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t nw = gridDim.x * wpg;
    const bool pack = h.sparse_packing == 2 || (h.sparse_packing == 1 && L.r > nw);
    const uint32_t nd = pack ? L.nd : L.r;       // items served one block per wavefront
    const uint32_t ns = L.r - nd;
    const uint32_t items = nd + (ns + 1) / 2;
    const uint32_t lane = lane_id();
    for (uint32_t item = xcd_logical_wg() * wpg + (threadIdx.x >> 6); item < items; item += nw) {
        uint32_t bid, slot = lane;
        bool live;
        const bool pair = item >= nd;
        if (!pair) {
            bid = __builtin_amdgcn_readfirstlane(L.at(item));
            const uint32_t t = __builtin_amdgcn_readfirstlane(h.type[bid]);
            const uint64_t bm = uniform64(walk_bitmaps(h, cls, snapshot)[bid]);
            live = t == cls && ((bm >> lane) & 1);
        } else {
            const uint32_t j = 2 * (item - nd) + (lane >> 5);
            const bool valid = j < ns;
            bid = L.R[L.M - 1 - (valid ? j : j - 1)];
            const uint64_t bm = walk_bitmaps(h, cls, snapshot)[bid];
            const uint32_t rank = lane & 31;
            live = valid && h.type[bid] == cls && rank < (uint32_t)__popcll(bm);
            slot = live ? nth_set_bit(bm, rank) : 0;
        }
        f(bid, slot, live, pair);
    }
}

// Releases the objects that delete themselves in a packed do-all (die on the
// lanes whose object is deleted; bid, slot and pair as for_each_object_packed
// passes them): one multi-slot release per block of the wavefront, the two
// blocks of a pair released side by side by lanes 0 and 32.  Converged call.
__device__ __forceinline__ void wave_release_packed(const HeapView &h, uint32_t cls, uint32_t bid, uint32_t slot,
                                                    bool die, bool pair)
{
    if (!pair) {
        wave_release_own_block(h, cls, bid, __ballot(die));
        return;
    }
    if (!__ballot(die)) return;
    // slot mask of each half's block: an OR over the 32 lanes of the half
    const uint64_t bit = die ? 1ull << slot : 0ull;
    uint32_t lo = (uint32_t)bit, hi = (uint32_t)(bit >> 32);
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        lo |= (uint32_t)__shfl_xor((int)lo, d);
        hi |= (uint32_t)__shfl_xor((int)hi, d);
    }
    const uint64_t mask = ((uint64_t)hi << 32) | lo;
    OpQueue q;
    q.reset();
    if ((lane_id() & 31) == 0 && mask) release_slots(h, cls, bid, mask, q);
    run_ops_wave(h, q);
}

template <class T>
__device__ __forceinline__ T *farr(const HeapView &h, uint32_t bid, uint32_t off)
{
    return reinterpret_cast<T *>(h.block(bid) + off);
}

template <class T>
__device__ __forceinline__ T &fref(const HeapView &h, uint32_t handle, uint32_t off)
{
    return reinterpret_cast<T *>(h.block(handle >> 6) + off)[handle & 63];
}

inline smmo_status launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SMMO_OK : hip_fail(e, what);
}

// Kernel parameters for (method tag, class, argument struct), bound by
// `bind` on the first launch and taken from the heap's cache afterwards.
template <class K, class A, class Bind>
smmo_status cached_bind(smmo_heap *h, const void *tag, uint32_t cls, const A &a, K &k, Bind &&bind)
{
    static_assert(sizeof(A) <= sizeof(smmo_bind_slot::args) && sizeof(K) <= sizeof(smmo_bind_slot::k),
                  "bind cache slot too small");
    for (smmo_bind_slot &sl : h->bind_cache)
        if (sl.method == tag && sl.cls == cls && sl.nargs == sizeof(A) && sl.nk == sizeof(K) &&
            memcmp(sl.args, &a, sizeof(A)) == 0) {
            memcpy(&k, sl.k, sizeof(K));
            return SMMO_OK;
        }
    smmo_status s = bind();
    if (s) return s;
    smmo_bind_slot &sl = h->bind_cache[h->bind_next++ % (sizeof(h->bind_cache) / sizeof(h->bind_cache[0]))];
    sl.method = tag;
    sl.cls = cls;
    sl.nargs = sizeof(A);
    sl.nk = sizeof(K);
    memcpy(sl.args, &a, sizeof(A));
    memcpy(sl.k, &k, sizeof(K));
    return SMMO_OK;
}

#define BIND(cls, name, dt, cnt, off, stride)                                              \
    do {                                                                                   \
        smmo_status _s = bind_field(h->schema, (cls), (name), (dt), (cnt), (off), (stride)); \
        if (_s) return _s;                                                                 \
    } while (0)

} // namespace smmo
