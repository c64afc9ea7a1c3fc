// Layout of an SMMO heap in device memory, shared by host and device code.
//
// The caller's buffer holds, in this order (each region 256-byte aligned):
//   control words    error word, event counters, enumeration counters
//   bitmaps          free, then allocated[c] and active[c] for every class;
//                    each a stack of levels of 64-bit containers
//   type[M]          class of each block (kNull while never initialized)
//   alloc_bm[M]      64-bit object allocation bitmap of each block
//   iter_bm[M]       64-bit object iteration bitmap of each block
//   R[classes][M]    block lists built by the enumeration pre-pass
//   claim[M]         block ids claimed by an ordered bulk allocation
//   blocks[M]        M equal blocks; a block is the data segment of up to 64
//                    objects of one class, one 64-entry array per field
// The thesis keeps the two object bitmaps and the type id inside each block
// (Ch.5 sec.5.2.1 "Block Structure"); here they are dense per-block arrays so
// that enumeration reads them contiguously and the data segment holds only
// field arrays.  What the allocator's correctness needs from the in-block
// placement (every block's bitmap is at the same, type-independent place) is
// kept.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smmo {

constexpr uint32_t kNull = 0xFFFFFFFFu;       // no object
constexpr uint32_t kNoBlock = 0xFFFFFFFFu;
constexpr uint32_t kMaxLevels = 6;
constexpr uint32_t kMaxClasses = 16;
constexpr uint32_t kMaxBlocks = (1u << 25) - 2;
// Event counters are striped: 64 stripes of 128 bytes each, a wavefront
// adds to stripe (its global wavefront id mod 64), so that concurrent
// allocations and deletions do not all hit one address; readers sum them.
constexpr uint32_t kEventStripes = 64;
constexpr uint32_t kStripeWords = 32;
constexpr uint32_t CTRL_EVENTS = 1024;        // first word of stripe 0
constexpr uint32_t kCtrlWords = CTRL_EVENTS + kEventStripes * kStripeWords;   // 12 KiB

constexpr uint32_t BM_FREE = 0;
__host__ __device__ constexpr uint32_t bm_alloc(uint32_t c) { return 1 + 2 * c; }
__host__ __device__ constexpr uint32_t bm_active(uint32_t c) { return 2 + 2 * c; }

// device error word bits
enum : uint32_t {
    ERR_NOMEM = 1u,       // heap exhausted
    ERR_SPIN = 2u,        // a retry loop exceeded its bound
    ERR_BADHANDLE = 4u,   // a handle that names no live object of the class
    ERR_INTERNAL = 8u,    // internal limit (e.g. too many queued bitmap switches)
};

// control word indices (uint32 units; 64-bit counters take two words)
enum : uint32_t {
    CTRL_ERR = 0,
    CTRL_GCOUNT = 8,      // gather: running output count
    CTRL_GDONE = 9,       // gather: finished wavefronts
    CTRL_RPACK = 16,      // [class] u64 (words 16 + 2 class): an enumeration's running
                          // dense count (bits 0-24), sparse count (25-49) and
                          // finished work-groups (50-63); zero between enumerations
    CTRL_RFINAL = 48,     // [class] length of R after the last enumeration
    CTRL_DCOUNT = 64,     // defragmentation: number of candidate blocks
    CTRL_DMOVED = 66,     // u64: defragmentation: objects moved
    CTRL_RSFINAL = 112,   // [class] sparse blocks (the back of R) after the last enumeration
    CTRL_STATS = 128,     // u64 statistics / invariant results (host reads)
};

// u64 event counters inside each stripe (word offsets)
enum : uint32_t {
    EV_SLOW = 0,          // blocks initialized by device allocation
    EV_RETRY = 2,         // failed slot reservations (retried)
    EV_NEWS = 4,          // objects created by device allocation
    EV_DELS = 6,          // objects released by device deallocation
    EV_SPIN = 8,          // extra rounds of converged bitmap switches
    EV_FIND = 10,         // active-block and free-block searches
};

// statistics block (u64 words starting at CTRL_STATS)
enum : uint32_t {
    ST_LIVE = 0,          // [class]
    ST_BLOCKS = 16,       // [class]
    ST_FREE = 32,
    ST_HIER = 33,
    ST_STATE = 34,
    ST_ACTIVE = 35,
    ST_TYPE = 36,
    ST_EMPTY = 37,
    ST_WORDS = 40,
};

// What a kernel needs to know about the heap; passed by value.
struct HeapView {
    char *blocks;
    uint64_t block_bytes;
    uint64_t *bm;                 // all bitmaps, bm_words each
    uint32_t *type;
    uint64_t *alloc_bm;
    uint64_t *iter_bm;
    uint32_t *R;                  // R + c * M is class c's block list
    uint32_t *claim;
    uint32_t *ctrl;
    uint32_t M;
    uint32_t nclasses;
    uint32_t nlev;                // levels per bitmap (level nlev-1 has one container)
    uint32_t bm_words;
    uint32_t lvl_off[kMaxLevels]; // word offset of each level inside a bitmap
    uint32_t lvl_n[kMaxLevels];   // containers per level
    uint32_t retries;
    uint32_t rotation;
    uint32_t coalescing;
    uint32_t spin_limit;
    uint32_t sparse_packing;      // 0 never, 1 when the list outgrows the grid, 2 always
    uint32_t direct;              // classes whose walks this launch visit every block (bit c = class c)
    uint32_t snap;                // classes whose walks this launch read the iteration bitmaps of a
                                  // snapshot taken earlier by smmo_snapshot (bit c = class c)

    __host__ __device__ uint64_t *bm_word(uint32_t bmid, uint32_t lvl, uint32_t c) const
    {
        return bm + (uint64_t)bmid * bm_words + lvl_off[lvl] + c;
    }
    __host__ __device__ char *block(uint32_t bid) const { return blocks + (uint64_t)bid * block_bytes; }
};

// The block list R of a class as the enumeration leaves it: its r entries are
// the dense blocks (more than 32 live objects when enumerated) from the front
// of the class's M-entry region, then the sparse blocks from the back.  A list
// stays in use until something may allocate objects of its class, so a block
// listed as sparse never holds more than 32 live objects while it is used
// (deletions only move blocks from dense towards sparse).
// A direct list (HeapView::direct) is every block of the heap, 0 .. M-1, in
// order: a walk that checks each block's type then visits the class's blocks
// without a list.  The host uses it in place of a stale list on small heaps,
// for walks that create no objects of the class they walk.
struct BlockList {
    const uint32_t *R;
    uint32_t r, nd, M, direct;
    __host__ __device__ uint32_t at(uint32_t i) const
    {
        return direct ? i : i < nd ? R[i] : R[M - 1 - (i - nd)];
    }
};

} // namespace smmo
