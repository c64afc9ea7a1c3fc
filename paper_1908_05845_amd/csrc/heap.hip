// libsmmo: schema, heap and SMMO operations (C ABI in include/smmo.h).
//
// Heap operations follow the DynaSOAr design (Springer, Ch.5): equal-size
// blocks of one class each, hierarchical block-state bitmaps, the lock-free
// object allocator, and do-all enumeration over a compacted list of
// allocated blocks (sec.5.2.7, with the bitmap `indices` operation of
// sec.5.3.1).  Device code is in smmo_device.hpp; methods in methods.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "smmo_device.hpp"
#include "smmo_host.hpp"

using namespace smmo;

namespace {

thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    uint32_t nlev = 0;
    uint32_t lvl_n[kMaxLevels] = {};
    uint32_t lvl_off[kMaxLevels] = {};
    uint32_t bm_words = 0;
    size_t ctrl = 0, bm = 0, type = 0, alloc = 0, iter = 0, R = 0, claim = 0, blocks = 0, total = 0;
};

void layout_for(uint32_t nclasses, uint64_t M, uint32_t block_bytes, Layout &L)
{
    L = Layout{};
    uint64_t n = (M + 63) / 64;
    uint32_t off = 0;
    for (;;) {
        L.lvl_n[L.nlev] = (uint32_t)n;
        L.lvl_off[L.nlev] = off;
        off += (uint32_t)n;
        L.nlev++;
        if (n == 1) break;
        n = (n + 63) / 64;
    }
    L.bm_words = off;
    const uint64_t nbm = 1 + 2ull * nclasses;
    size_t p = 0;
    L.ctrl = p;   p += align256(kCtrlWords * 4);
    L.bm = p;     p += align256(nbm * L.bm_words * 8);
    L.type = p;   p += align256(M * 4);
    L.alloc = p;  p += align256(M * 8);
    L.iter = p;   p += align256(M * 8);
    L.R = p;      p += align256((size_t)nclasses * M * 4);
    L.claim = p;  p += align256(M * 4);
    L.blocks = p; p += (size_t)M * block_bytes;
    L.total = p;
}

uint32_t schema_block_bytes(const smmo_schema *s)
{
    uint32_t b = 256;
    for (uint32_t c = 0; c < s->nclasses; ++c) b = std::max(b, s->c[c].data_bytes);
    return b;
}

bool heap_ok(const smmo_heap *h) { return h && h->schema && h->base; }

smmo_status check_class(const smmo_heap *h, uint32_t cls)
{
    if (!heap_ok(h)) return fail(SMMO_EINVAL, "heap is NULL or freed");
    if (cls >= h->schema->nclasses) return fail(SMMO_EINVAL, "class id out of range");
    return SMMO_OK;
}

// ----------------------------------------------------------------- kernels --

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(v, (unsigned)d);
        if (lane >= (uint32_t)d) v += y;
    }
    return v;
}

// exclusive scan over a work-group of up to 1024 threads; *total = sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &total)
{
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t i = 0; i < nw; ++i) {
        const uint32_t x = s_w[i];
        if (i < w) before += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return before + incl - v;
}

// All blocks free (free bitmap full, allocation bitmaps all-ones as if
// invalidated, type unset), other bitmaps empty, control words zero.
__global__ void k_heap_init(HeapView h)
{
    const uint64_t nbw = (1ull + 2ull * h.nclasses) * h.bm_words;
    const uint64_t total = std::max<uint64_t>(std::max<uint64_t>(h.M, nbw), kCtrlWords);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (i < h.M) {
            h.type[i] = kNull;
            h.alloc_bm[i] = ~0ull;
            h.iter_bm[i] = 0;
        }
        if (i < nbw) {
            const uint32_t bmid = (uint32_t)(i / h.bm_words);
            const uint32_t w = (uint32_t)(i % h.bm_words);
            uint64_t val = 0;
            if (bmid == BM_FREE) {
                uint32_t l = 0;
                while (l + 1 < h.nlev && w >= h.lvl_off[l + 1]) ++l;
                const uint32_t c = w - h.lvl_off[l];
                const uint64_t nchild = l == 0 ? h.M : h.lvl_n[l - 1];
                const uint64_t lo = (uint64_t)c * 64;
                const uint64_t cnt = nchild > lo ? std::min<uint64_t>(64, nchild - lo) : 0;
                val = cnt == 64 ? ~0ull : ((1ull << cnt) - 1);
            }
            h.bm[i] = val;
        }
        if (i < kCtrlWords) h.ctrl[i] = 0;
    }
}

// Enumeration pre-pass (sec.5.2.7 with Alg. indices of sec.5.3.1): compact
// the set bits of allocated[cls] into R.  Work-group g owns level-0
// containers 1024 g .. 1024 g + 1023 (thread t loads container 1024 g + t,
// in the same batch of loads as the error word: the level-1 summary would
// only add a dependent load, and reading every container costs 8 bytes per
// 64 blocks).  Each group reserves its ranges of R (dense blocks at the
// front, sparse ones at the back) and counts itself finished with one 64-bit
// atomic add on the class's packed counter, so R is ordered within a
// group's ranges only.  The group whose add finds every other group
// finished knows the totals: it publishes the lengths and zeroes the
// counter, so the pass needs no reset launch and can be captured in a
// graph.  (The lengths are read by later launches only, after every group's
// appends have been performed.)
constexpr uint64_t kPackMask = (1ull << 25) - 1;
static_assert(kMaxBlocks <= kPackMask, "block counts must fit the packed enumeration counter");
static_assert((kMaxBlocks / 64 + 1024) / 1024 < (1u << 14), "work-group counts must fit the packed enumeration counter");

__global__ __launch_bounds__(1024) void k_enumerate(HeapView h, uint32_t cls, uint32_t snapshot, uint32_t split)
{
    const uint32_t lane = lane_id();
    const uint32_t wig = threadIdx.x >> 6;
    const uint32_t n0 = h.lvl_n[0];
    const uint32_t cidx = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t err = ald32(h.ctrl + CTRL_ERR);
    uint64_t c = cidx < n0 ? ald(h.bm_word(bm_alloc(cls), 0, cidx)) : 0ull;
    if (err) c = 0;       // a failed heap lists nothing
    // The packing plan (split): blocks with more than 32 live objects are
    // dense.  Without it every block counts as dense.  No wavefront changes
    // a bitmap while this kernel runs, so plain loads are enough.  The
    // per-block work (the snapshot copy, the plan) is spread over the
    // work-group: container j of the group's 1,024 goes to wave j mod 16,
    // one block per lane, so a lane issues its (at most 64) bitmap loads
    // eight at a time, independent of each other, instead of following one
    // container's set bits in a chain of dependent loads.
    __shared__ uint64_t s_c[1024], s_d[1024];
    __shared__ uint32_t s_nd[16], s_ns[16];
    __shared__ uint64_t s_old;
    uint64_t dense = c;
    if (snapshot || split) {
        s_c[threadIdx.x] = c;
        s_d[threadIdx.x] = 0;
        __syncthreads();
        const uint64_t gbase = (uint64_t)blockIdx.x * 1024 * 64;   // first block of the group
        const uint64_t *abm = h.alloc_bm + gbase;
        uint64_t *ibm = h.iter_bm + gbase;
        for (uint32_t j0 = wig; j0 < 1024; j0 += 128) {
            uint64_t cw[8], bm[8];
            uint64_t any = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cw[u] = s_c[j0 + 16 * u];
                any |= cw[u];
            }
            if (!any) continue;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                bm[u] = ((cw[u] >> lane) & 1) ? abm[(uint64_t)(j0 + 16 * u) * 64 + lane] : 0ull;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = (cw[u] >> lane) & 1;
                if (snapshot && in) ibm[(uint64_t)(j0 + 16 * u) * 64 + lane] = bm[u];
                const uint64_t d = __ballot(in && (!split || __popcll(bm[u]) > 32));
                if (lane == 0) s_d[j0 + 16 * u] = d;
            }
        }
        __syncthreads();
        dense = s_d[threadIdx.x];
    }
    const uint32_t nd = (uint32_t)__popcll(dense), ns = (uint32_t)__popcll(c) - nd;
    const uint32_t incl_d = wave_incl_scan(nd), incl_s = wave_incl_scan(ns);
    if (lane == 63) {
        s_nd[wig] = incl_d;
        s_ns[wig] = incl_s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t td = 0, ts = 0;
        for (int k = 0; k < 16; ++k) {
            td += s_nd[k];
            ts += s_ns[k];
        }
        const uint64_t add = (uint64_t)td | ((uint64_t)ts << 25) | (1ull << 50);
        uint64_t *pack = reinterpret_cast<uint64_t *>(h.ctrl + CTRL_RPACK + 2 * cls);
        const uint64_t old = __hip_atomic_fetch_add(pack, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_old = old;
        if ((old >> 50) == gridDim.x - 1) {
            const uint64_t tot = old + add;
            const uint32_t rd = (uint32_t)(tot & kPackMask), rs = (uint32_t)((tot >> 25) & kPackMask);
            __hip_atomic_store(h.ctrl + CTRL_RFINAL + cls, rd + rs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(h.ctrl + CTRL_RSFINAL + cls, rs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pack, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    const uint64_t old = s_old;
    uint32_t kd = (uint32_t)(old & kPackMask) + incl_d - nd, ks = (uint32_t)((old >> 25) & kPackMask) + incl_s - ns;
    for (uint32_t k = 0; k < wig; ++k) {      // the ranges of the group's earlier wavefronts
        kd += s_nd[k];
        ks += s_ns[k];
    }
    uint32_t *R = h.R + (uint64_t)cls * h.M;
    for (; c; c &= c - 1) {
        const uint32_t b = (uint32_t)(__ffsll((unsigned long long)c) - 1);
        if ((dense >> b) & 1) R[kd++] = cidx * 64 + b;
        else R[h.M - 1 - ks++] = cidx * 64 + b;
    }
}

struct FieldCopy {
    uint32_t offset;     // byte offset of element 0's array in a block
    uint32_t stride;     // bytes between inner elements' arrays
    uint32_t size;       // bytes per element (1 or 4)
    uint32_t count;      // inner elements
    const void *src;     // dense source (NULL = zero fill), or destination for gather
};

struct FieldSet {
    uint32_t nf;
    FieldCopy f[SMMO_MAX_FIELDS];
};

__device__ __forceinline__ void init_object(const HeapView &h, const FieldSet &fs, uint32_t handle,
                                            uint64_t i)
{
    char *base = h.block(handle >> 6);
    const uint32_t slot = handle & 63;
    for (uint32_t f = 0; f < fs.nf; ++f) {
        const FieldCopy &fc = fs.f[f];
        for (uint32_t q = 0; q < fc.count; ++q) {
            char *dst = base + fc.offset + q * fc.stride + slot * fc.size;
            const uint64_t e = i * fc.count + q;
            if (fc.size == 4) {
                *reinterpret_cast<uint32_t *>(dst) =
                    fc.src ? reinterpret_cast<const uint32_t *>(fc.src)[e] : 0u;
            } else {
                *reinterpret_cast<uint8_t *>(dst) =
                    fc.src ? reinterpret_cast<const uint8_t *>(fc.src)[e] : (uint8_t)0;
            }
        }
    }
}

// Ordered bulk claim for parallel_new: one work-group takes the `need` lowest
// free blocks in ascending order, clears their free bits, recomputes the free
// bitmap's summary levels over the touched range, and marks the blocks as
// allocated (and the last one active when it is only partly filled).  Runs
// while no other kernel uses the heap (calls on a heap are stream-ordered),
// so plain read-modify-write suffices.
__global__ __launch_bounds__(1024) void k_bulk_claim(HeapView h, uint32_t cls, uint32_t need,
                                                     uint32_t partial)
{
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_lo, s_hi;
    if (heap_failed(h)) return;
    const uint32_t t = threadIdx.x;
    const uint32_t n0 = h.lvl_n[0];
    uint64_t *F0 = h.bm_word(BM_FREE, 0, 0);

    uint32_t cnt = 0;
    for (uint32_t c = t; c < n0; c += blockDim.x) cnt += (uint32_t)__popcll(F0[c]);
    uint32_t total;
    block_excl_scan(cnt, s_w, total);
    if (total < need) {
        if (t == 0) raise_error(h, ERR_NOMEM);
        return;
    }
    if (t == 0) {
        s_lo = 0xFFFFFFFFu;
        s_hi = 0;
    }
    __syncthreads();
    uint32_t found = 0;
    for (uint32_t base = 0; base < n0 && found < need; base += blockDim.x) {
        const uint32_t c = base + t;
        const uint64_t v = c < n0 ? F0[c] : 0ull;
        const uint32_t k = (uint32_t)__popcll(v);
        uint32_t T;
        const uint32_t p = block_excl_scan(k, s_w, T);
        if (k && found + p < need) {
            const uint32_t take = std::min(k, need - found - p);
            const uint64_t taken = lowest_bits(v, take);
            F0[c] = v & ~taken;
            // the container's blocks join allocated[cls] with one OR per level
            aor(h.bm_word(bm_alloc(cls), 0, c), taken);
            for (uint32_t l = 1; l < h.nlev; ++l)
                aor(h.bm_word(bm_alloc(cls), l, c >> (6 * l)), 1ull << ((c >> (6 * (l - 1))) & 63));
            uint32_t o = found + p;
            for (uint64_t bits = taken; bits; bits &= bits - 1)
                h.claim[o++] = c * 64 + (uint32_t)(__ffsll((unsigned long long)bits) - 1);
            atomicMin(&s_lo, c);
            atomicMax(&s_hi, c);
        }
        found += T;
    }
    __syncthreads();
    uint32_t lo = s_lo, hi = s_hi;
    for (uint32_t l = 1; l < h.nlev; ++l) {
        lo >>= 6;
        hi >>= 6;
        for (uint32_t j = lo + t; j <= hi; j += blockDim.x) {
            uint64_t v = 0;
            for (uint32_t b = 0; b < 64; ++b) {
                const uint32_t child = j * 64 + b;
                if (child < h.lvl_n[l - 1] && *h.bm_word(BM_FREE, l - 1, child) != 0) v |= 1ull << b;
            }
            *h.bm_word(BM_FREE, l, j) = v;
        }
        __syncthreads();
    }
    // the partly filled last block is active (it has free slots)
    if (partial && t == 0) {
        uint32_t pos = h.claim[need - 1];
        for (uint32_t l = 0; l < h.nlev; ++l, pos >>= 6)
            aor(h.bm_word(bm_active(cls), l, pos >> 6), 1ull << (pos & 63));
    }
}

// Block headers of the claimed blocks (type, allocation bitmap): one thread
// per block, any number of work-groups.  The heap is quiescent during a bulk
// parallel_new, so the launch boundaries order these stores against the
// bitmaps written by k_bulk_claim.
__global__ __launch_bounds__(256) void k_bulk_headers(HeapView h, uint32_t cls, uint32_t need, uint32_t partial)
{
    if (heap_failed(h)) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < need; i += gridDim.x * blockDim.x) {
        const uint32_t bid = h.claim[i];
        const bool full = !(partial && i == need - 1);
        h.type[bid] = cls;
        h.alloc_bm[bid] = full ? ~0ull : ((1ull << partial) - 1);
    }
}

// Fills the objects of an ordered bulk claim: object i -> block claim[i/64],
// slot i%64 (64 consecutive objects share a block, so every field write of a
// wavefront is one contiguous run).
__global__ __launch_bounds__(256) void k_bulk_init(HeapView h, FieldSet fs, uint32_t n,
                                                   uint32_t *out_handles)
{
    if (heap_failed(h)) return;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t handle = (h.claim[i >> 6] << 6) | (uint32_t)(i & 63);
    init_object(h, fs, handle, i);
    if (out_handles) out_handles[i] = handle;
}

// parallel_new through the device allocator: every object is allocated by
// wavefront-aggregated device new (Alg. allocate with request coalescing)
// and then initialized, as in the thesis's parallel_new kernel.
__global__ __launch_bounds__(256) void k_new_device(HeapView h, uint32_t cls, FieldSet fs, uint32_t n,
                                                    uint32_t *out_handles)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (heap_failed(h)) return;                // uniform: one word for everyone
    const bool want = i < n;
    const uint32_t handle = wave_allocate(h, cls, want);
    if (!want) return;
    if (handle != kNull) init_object(h, fs, handle, i);
    if (out_handles) out_handles[i] = handle;
}

// Host-initiated destroy: validates each handle (live object of the class)
// and releases it through the converged deallocation path.
__global__ __launch_bounds__(256) void k_destroy(HeapView h, uint32_t cls, const uint32_t *handles,
                                                 uint32_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (heap_failed(h)) return;
    bool want = false;
    uint32_t hd = kNull;
    if (i < n) {
        hd = handles[i];
        const uint32_t bid = hd >> 6;
        want = hd != kNull && bid < h.M && ald32(h.type + bid) == cls &&
               ((ald(h.alloc_bm + bid) >> (hd & 63)) & 1);
        if (!want) raise_error(h, ERR_BADHANDLE);
    }
    wave_deallocate(h, cls, hd, want);
}

// Copies fields of the live objects (block by block, in R order) into dense
// arrays; the last wavefront publishes the count.
__global__ __launch_bounds__(256) void k_gather(HeapView h, uint32_t cls, FieldSet fs,
                                                uint32_t *out_handles, uint32_t capacity,
                                                uint32_t *out_count)
{
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    if (!heap_failed(h)) {
        const BlockList L = block_list(h, cls);
        for (uint32_t i = global_wave_id(); i < L.r; i += nw) {
            const uint32_t bid = L.at(i);
            if (ald32(h.type + bid) != cls) continue;
            const uint64_t bm = ald(h.alloc_bm + bid);
            const uint32_t cnt = (uint32_t)__popcll(bm);
            uint32_t base = 0;
            if (lane == 0)
                base = __hip_atomic_fetch_add(h.ctrl + CTRL_GCOUNT, cnt, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            base = __shfl(base, 0);
            if (!((bm >> lane) & 1)) continue;
            const uint64_t idx = base + (uint32_t)__popcll(bm & ((1ull << lane) - 1));
            if (idx >= capacity) continue;
            const char *src = h.block(bid);
            for (uint32_t f = 0; f < fs.nf; ++f) {
                const FieldCopy &fc = fs.f[f];
                for (uint32_t q = 0; q < fc.count; ++q) {
                    const char *s = src + fc.offset + q * fc.stride + lane * fc.size;
                    char *d = (char *)fc.src + (idx * fc.count + q) * fc.size;
                    if (fc.size == 4)
                        *reinterpret_cast<uint32_t *>(d) = *reinterpret_cast<const uint32_t *>(s);
                    else
                        *reinterpret_cast<uint8_t *>(d) = *reinterpret_cast<const uint8_t *>(s);
                }
            }
            if (out_handles) out_handles[idx] = (bid << 6) | lane;
        }
    }
    if (lane == 0) {
        const uint32_t d = __hip_atomic_fetch_add(h.ctrl + CTRL_GDONE, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (d == nw - 1) {
            *out_count = ald32(h.ctrl + CTRL_GCOUNT);
            __hip_atomic_store(h.ctrl + CTRL_GCOUNT, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(h.ctrl + CTRL_GDONE, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_zero_words(uint32_t *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__device__ __forceinline__ bool bm_bit(const HeapView &h, uint32_t bmid, uint32_t pos)
{
    return (ald(h.bm_word(bmid, 0, pos >> 6)) >> (pos & 63)) & 1;
}

// Statistics and invariant check of a quiescent heap.
__global__ __launch_bounds__(256) void k_stats(HeapView h)
{
    unsigned long long *st = reinterpret_cast<unsigned long long *>(h.ctrl + CTRL_STATS);
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = gid; b < h.M; b += gsz) {
        const uint32_t bid = (uint32_t)b;
        const bool fr = bm_bit(h, BM_FREE, bid);
        const uint32_t t = h.type[bid];
        const uint64_t bm = h.alloc_bm[bid];
        uint32_t nalloc = 0;
        for (uint32_t c = 0; c < h.nclasses; ++c) {
            const bool a = bm_bit(h, bm_alloc(c), bid);
            const bool act = bm_bit(h, bm_active(c), bid);
            if (a) {
                nalloc++;
                if (t != c) {
                    atomicAdd(st + ST_TYPE, 1ull);
                } else {
                    atomicAdd(st + ST_LIVE + c, (unsigned long long)__popcll(bm));
                    atomicAdd(st + ST_BLOCKS + c, 1ull);
                    if (bm == 0) atomicAdd(st + ST_EMPTY, 1ull);
                    if (act != (bm != ~0ull)) atomicAdd(st + ST_ACTIVE, 1ull);
                }
            } else if (act) {
                atomicAdd(st + ST_ACTIVE, 1ull);
            }
        }
        if (fr) {
            atomicAdd(st + ST_FREE, 1ull);
            if (nalloc || t != kNull) atomicAdd(st + ST_STATE, 1ull);
        } else if (nalloc != 1) {
            atomicAdd(st + ST_STATE, 1ull);
        }
    }
    // container consistency of every summary level, and no bits past the end
    const uint64_t nbm = 1ull + 2ull * h.nclasses;
    const uint64_t words = nbm * h.bm_words;
    for (uint64_t i = gid; i < words; i += gsz) {
        const uint32_t bmid = (uint32_t)(i / h.bm_words);
        const uint32_t w = (uint32_t)(i % h.bm_words);
        uint32_t l = 0;
        while (l + 1 < h.nlev && w >= h.lvl_off[l + 1]) ++l;
        const uint32_t c = w - h.lvl_off[l];
        const uint64_t actual = h.bm[i];
        const uint64_t nchild = l == 0 ? h.M : h.lvl_n[l - 1];
        uint64_t expect_mask = ~0ull;
        const uint64_t lo = (uint64_t)c * 64;
        const uint64_t cnt = nchild > lo ? std::min<uint64_t>(64, nchild - lo) : 0;
        if (cnt < 64) expect_mask = (1ull << cnt) - 1;
        bool bad = (actual & ~expect_mask) != 0;
        if (l > 0) {
            uint64_t expect = 0;
            for (uint32_t b = 0; b < cnt; ++b)
                if (*h.bm_word(bmid, l - 1, c * 64 + b) != 0) expect |= 1ull << b;
            bad |= expect != actual;
        }
        if (bad) atomicAdd(st + ST_HIER, 1ull);
    }
}

smmo_status launch_check(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return SMMO_OK;
}

smmo_status build_fieldset(const smmo_heap *h, uint32_t cls, const uint32_t *ids, uint32_t n,
                           const void *const *ptrs, FieldSet &fs)
{
    const smmo_class_info &ci = h->schema->c[cls];
    fs.nf = n;
    for (uint32_t j = 0; j < n; ++j) {
        if (ids[j] >= ci.nfields) return fail(SMMO_EINVAL, "field id out of range");
        for (uint32_t k = 0; k < j; ++k)
            if (ids[k] == ids[j]) return fail(SMMO_EINVAL, "field listed twice");
        const smmo_field_info &fi = ci.f[ids[j]];
        fs.f[j] = FieldCopy{fi.offset, fi.stride, fi.size, fi.count, ptrs ? ptrs[j] : nullptr};
    }
    return SMMO_OK;
}

smmo_status read_ctrl(smmo_heap *h, uint32_t first_word, uint32_t nwords)
{
    hipError_t e = hipStreamSynchronize(h->last);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipMemcpy(reinterpret_cast<char *>(h->host_ctrl) + first_word * 4,
                  h->v.ctrl + first_word, (size_t)nwords * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(control words)");
    return SMMO_OK;
}

smmo_status map_device_error(uint32_t err)
{
    if (!err) return SMMO_OK;
    if (err == ERR_NOMEM) return fail(SMMO_ENOMEM, "device: heap exhausted during allocation");
    std::string m = "device error:";
    if (err & ERR_NOMEM) m += " heap exhausted;";
    if (err & ERR_SPIN) m += " retry bound exceeded;";
    if (err & ERR_BADHANDLE) m += " handle not a live object of the class;";
    if (err & ERR_INTERNAL) m += " internal limit;";
    return fail(SMMO_EDEVICE, m);
}

smmo_status run_stats(smmo_heap *h, hipStream_t st)
{
    const uint32_t nw = ST_WORDS * 2;
    hipLaunchKernelGGL(k_zero_words, dim3((nw + 255) / 256), dim3(256), 0, st,
                       h->v.ctrl + CTRL_STATS, nw);
    const uint64_t work = std::max<uint64_t>(h->v.M, (1ull + 2ull * h->v.nclasses) * h->v.bm_words);
    const uint32_t grid = (uint32_t)std::min<uint64_t>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_stats, dim3(grid), dim3(256), 0, st, h->v);
    smmo_status s = launch_check("k_stats");
    if (s) return s;
    h->last = st;
    return read_ctrl(h, 0, kCtrlWords);
}

} // namespace

// ------------------------------------------------------- internal helpers --
namespace smmo {

smmo_status heap_check_class(const smmo_heap *h, uint32_t cls) { return check_class(h, cls); }
smmo_status heap_read_ctrl(smmo_heap *h, uint32_t first_word, uint32_t nwords)
{
    return read_ctrl(h, first_word, nwords);
}
smmo_status heap_launch_check(const char *what) { return launch_check(what); }

smmo_status fail(smmo_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

smmo_status hip_fail(hipError_t e, const char *what)
{
    return fail(SMMO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint32_t dtype_size(int32_t dtype)
{
    switch (dtype) {
    case SMMO_U8: return 1;
    case SMMO_I32:
    case SMMO_U32:
    case SMMO_F32:
    case SMMO_HANDLE: return 4;
    default: return 0;
    }
}

smmo_status bind_field(const smmo_schema *s, uint32_t cls, const char *name, int32_t dtype,
                       uint32_t count, uint32_t *offset, uint32_t *stride)
{
    if (cls >= s->nclasses) return fail(SMMO_EINVAL, "class id out of range");
    const smmo_class_info &ci = s->c[cls];
    for (uint32_t j = 0; j < ci.nfields; ++j) {
        const smmo_field_info &f = ci.f[j];
        if (strcmp(f.name, name) != 0) continue;
        if (f.dtype != dtype || (count && f.count != count))
            return fail(SMMO_EINVAL, std::string("class '") + ci.name + "': field '" + name +
                                         "' has the wrong type or length for this method");
        *offset = f.offset;
        if (stride) *stride = f.stride;
        return SMMO_OK;
    }
    return fail(SMMO_EINVAL, std::string("class '") + ci.name + "' has no field '" + name +
                                 "' required by this method");
}

smmo_status ensure_enumerated(smmo_heap *h, uint32_t cls, bool snapshot, hipStream_t st, bool split,
                              bool allow_direct)
{
    // a do-all that uses a snapshot from smmo_snapshot walks that list as it is
    if ((h->v.snap >> cls) & 1) return SMMO_OK;
    if (!snapshot && (h->rstate[cls] == R_SPLIT || (h->rstate[cls] == R_VALID && !split))) return SMMO_OK;
    // A walk that needs neither the iteration snapshot nor the packing plan
    // reads nothing of R but its entries; on a small heap the walk over all
    // blocks costs less than the enumeration launch it replaces, for a class
    // whose list goes stale at every launch that creates its objects.  The
    // list stays stale (rstate unchanged); every such launch walks directly.
    if (allow_direct && !snapshot && !split && h->churn[cls] && h->v.M <= kDirectMaxBlocks) {
        h->v.direct |= 1u << cls;
        return SMMO_OK;
    }
    h->v.direct &= ~(1u << cls);
    h->snap_pending &= ~(1u << cls);     // the list is rebuilt: a snapshot taken before is gone
    const uint32_t nwaves = (h->v.lvl_n[0] + 63) / 64;
    const uint32_t grid = (nwaves + 15) / 16;
    hipLaunchKernelGGL(k_enumerate, dim3(grid), dim3(1024), 0, st, h->v, cls, snapshot ? 1u : 0u,
                       split ? 1u : 0u);
    smmo_status s = launch_check("k_enumerate");
    if (s) return s;
    h->rstate[cls] = split ? R_SPLIT : R_VALID;
    return SMMO_OK;
}

bool packing_wanted(const smmo_heap *h, uint32_t cls, const LaunchShape &ls)
{
    const uint64_t waves = (uint64_t)ls.grid.x * (ls.block.x / 64);
    return h->cfg.sparse_packing == 2 || (h->cfg.sparse_packing == 1 && h->ub_blocks[cls] > waves);
}

LaunchShape method_shape(const smmo_heap *h, uint32_t cls, uint32_t def_group)
{
    uint32_t wg = 256;
    uint64_t waves = h->cfg.grid_waves ? h->cfg.grid_waves : 64ull * h->cu_count;
    uint32_t group = def_group == 0 ? 1 : h->cfg.block_group ? h->cfg.block_group : def_group;
    if (h->cur_method < 64) {
        if (h->launch_wg[h->cur_method][cls]) wg = h->launch_wg[h->cur_method][cls];
        if (h->launch_waves[h->cur_method][cls]) waves = h->launch_waves[h->cur_method][cls];
        if (def_group && h->launch_group[h->cur_method][cls]) group = h->launch_group[h->cur_method][cls];
    }
    const uint64_t groups = (std::max<uint64_t>(1, h->ub_blocks[cls]) + group - 1) / group;
    waves = std::min<uint64_t>(waves, groups);
    const uint32_t wpg = wg / 64;
    LaunchShape ls;
    ls.grid = dim3((uint32_t)((waves + wpg - 1) / wpg));
    ls.block = dim3(wg);
    ls.group = group;
    return ls;
}

uint32_t class_family(const smmo_schema *s, uint32_t cls)
{
    uint32_t fam = 0;
    for (uint32_t c = 0; c < s->nclasses; ++c)
        for (uint32_t a = c; a != SMMO_NO_PARENT; a = s->c[a].parent)
            if (a == cls) {
                fam |= 1u << c;
                break;
            }
    return fam;
}

void note_allocation(smmo_heap *h, uint32_t cls, uint64_t max_new_objects, bool in_method)
{
    if (in_method) h->churn[cls] = true;
    const uint64_t add = (max_new_objects + 63) / 64 + 1;
    h->ub_blocks[cls] = std::min<uint64_t>(h->v.M, h->ub_blocks[cls] + add);
    h->rstate[cls] = R_DIRTY;
}

} // namespace smmo

// ===================================================================== ABI ==
extern "C" {

void smmo_config_default(smmo_config *cfg)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof *cfg);
    cfg->lookup_retries = 5;
    cfg->rotation = 1;
    cfg->coalescing = 1;
    cfg->bulk_ordered = 1;
    cfg->spin_limit = 1u << 20;
    cfg->grid_waves = 0;
}

smmo_status smmo_schema_create(smmo_schema **out)
{
    if (!out) return fail(SMMO_EINVAL, "out is NULL");
    *out = new (std::nothrow) smmo_schema();
    return *out ? SMMO_OK : fail(SMMO_ENOMEM, "host allocation failed");
}

smmo_status smmo_schema_free(smmo_schema *s)
{
    delete s;
    return SMMO_OK;
}

smmo_status smmo_define_class(smmo_schema *s, const char *name, const smmo_field_desc *fields,
                              uint32_t nfields, uint32_t *class_id)
{
    if (!fields) return fail(SMMO_EINVAL, "NULL argument");
    return smmo_define_subclass(s, name, SMMO_NO_PARENT, 0, fields, nfields, class_id);
}

smmo_status smmo_define_subclass(smmo_schema *s, const char *name, uint32_t parent, uint32_t flags,
                                 const smmo_field_desc *fields, uint32_t nfields, uint32_t *class_id)
{
    if (!s || !name || !class_id || (nfields && !fields)) return fail(SMMO_EINVAL, "NULL argument");
    if (s->frozen) return fail(SMMO_ESTATE, "schema is frozen: a heap was created from it");
    if (s->nclasses >= SMMO_MAX_CLASSES) return fail(SMMO_ENOMEM, "too many classes");
    if (flags & ~SMMO_CLASS_ABSTRACT) return fail(SMMO_EINVAL, "unknown class flags");
    if (parent != SMMO_NO_PARENT && parent >= s->nclasses) return fail(SMMO_EINVAL, "parent class id out of range");
    const size_t nl = strlen(name);
    if (nl == 0 || nl > 31) return fail(SMMO_EINVAL, "class name must have 1..31 characters");
    for (uint32_t c = 0; c < s->nclasses; ++c)
        if (strcmp(s->c[c].name, name) == 0) return fail(SMMO_EINVAL, "duplicate class name");
    // the inherited fields first (same order, hence the same offsets), then the new ones
    smmo_field_desc all[SMMO_MAX_FIELDS];
    uint32_t ninh = 0;
    if (parent != SMMO_NO_PARENT) {
        const smmo_class_info &pc = s->c[parent];
        for (uint32_t j = 0; j < pc.nfields; ++j)
            all[ninh++] = smmo_field_desc{pc.f[j].name, pc.f[j].dtype, pc.f[j].count};
    }
    if (nfields > SMMO_MAX_FIELDS - ninh) return fail(SMMO_EINVAL, "bad field count");
    for (uint32_t j = 0; j < nfields; ++j) all[ninh + j] = fields[j];
    nfields += ninh;
    if (nfields == 0) return fail(SMMO_EINVAL, "bad field count");
    smmo_class_info ci{};
    memcpy(ci.name, name, nl + 1);
    ci.nfields = nfields;
    ci.parent = parent;
    ci.flags = flags;
    uint32_t cur = 0, arrays = 0;
    for (uint32_t j = 0; j < nfields; ++j) {
        const smmo_field_desc &fd = all[j];
        if (!fd.name) return fail(SMMO_EINVAL, "field name is NULL");
        const size_t fl = strlen(fd.name);
        if (fl == 0 || fl > 31) return fail(SMMO_EINVAL, "field name must have 1..31 characters");
        for (uint32_t k = 0; k < j; ++k)
            if (strcmp(ci.f[k].name, fd.name) == 0) return fail(SMMO_EINVAL, "duplicate field name");
        const uint32_t sz = dtype_size(fd.dtype);
        if (!sz) return fail(SMMO_EINVAL, std::string("field '") + fd.name + "': bad dtype");
        if (fd.count == 0) return fail(SMMO_EINVAL, std::string("field '") + fd.name + "': count 0");
        arrays += fd.count;
        if (arrays > SMMO_MAX_FIELDS) return fail(SMMO_EINVAL, "too many field arrays in class");
        smmo_field_info &fi = ci.f[j];
        memcpy(fi.name, fd.name, fl + 1);
        fi.dtype = fd.dtype;
        fi.count = fd.count;
        fi.size = sz;
        // one 64-entry array per element, aligned to its own size (<= 256 B)
        const uint32_t arr = SMMO_BLOCK_CAPACITY * sz;
        const uint32_t al = std::min<uint32_t>(256, arr);
        cur = (cur + al - 1) / al * al;
        fi.offset = cur;
        fi.stride = (arr + al - 1) / al * al;
        cur += fi.stride * fd.count;
    }
    ci.narrays = arrays;
    ci.data_bytes = (uint32_t)align256(cur);
    s->c[s->nclasses] = ci;
    *class_id = s->nclasses++;
    return SMMO_OK;
}

smmo_status smmo_class_is_a(const smmo_schema *s, uint32_t cls, uint32_t ancestor, uint32_t *out)
{
    if (!s || !out) return fail(SMMO_EINVAL, "NULL argument");
    if (cls >= s->nclasses || ancestor >= s->nclasses) return fail(SMMO_EINVAL, "class id out of range");
    *out = (smmo::class_family(s, ancestor) >> cls) & 1u;
    return SMMO_OK;
}

smmo_status smmo_field_id(const smmo_schema *s, uint32_t class_id, const char *name, uint32_t *field_id)
{
    if (!s || !name || !field_id) return fail(SMMO_EINVAL, "NULL argument");
    if (class_id >= s->nclasses) return fail(SMMO_EINVAL, "class id out of range");
    const smmo_class_info &ci = s->c[class_id];
    for (uint32_t j = 0; j < ci.nfields; ++j)
        if (strcmp(ci.f[j].name, name) == 0) {
            *field_id = j;
            return SMMO_OK;
        }
    return fail(SMMO_EINVAL, std::string("no field '") + name + "'");
}

smmo_status smmo_block_bytes(const smmo_schema *s, uint32_t *block_bytes)
{
    if (!s || !block_bytes) return fail(SMMO_EINVAL, "NULL argument");
    if (!s->nclasses) return fail(SMMO_ESTATE, "schema has no classes");
    *block_bytes = schema_block_bytes(s);
    return SMMO_OK;
}

smmo_status smmo_heap_bytes(const smmo_schema *s, uint64_t blocks, uint64_t *bytes)
{
    if (!s || !bytes) return fail(SMMO_EINVAL, "NULL argument");
    if (!s->nclasses) return fail(SMMO_ESTATE, "schema has no classes");
    if (blocks == 0 || blocks > kMaxBlocks) return fail(SMMO_EINVAL, "block count out of range");
    Layout L;
    layout_for(s->nclasses, blocks, schema_block_bytes(s), L);
    *bytes = L.total;
    return SMMO_OK;
}

namespace {
std::mutex allocator_mu;
smmo_allocator allocator_set{};   // alloc == nullptr: none

smmo_status create_heap(smmo_schema *s, void *dev_buf, size_t bytes, const smmo_config *cfg, smmo_stream stream,
                        smmo_heap **out);
} // namespace

smmo_status smmo_set_allocator(const smmo_allocator *a)
{
    if (a && (!a->alloc || !a->release)) return fail(SMMO_EINVAL, "allocator: alloc and release must be set");
    std::lock_guard<std::mutex> lock(allocator_mu);
    allocator_set = a ? *a : smmo_allocator{};
    return SMMO_OK;
}

smmo_status smmo_alloc_heap(smmo_schema *s, void *dev_buf, size_t bytes, const smmo_config *cfg,
                            smmo_stream stream, smmo_heap **out)
{
    if (!s || !out) return fail(SMMO_EINVAL, "NULL argument");
    if (dev_buf) return create_heap(s, dev_buf, bytes, cfg, stream, out);
    smmo_allocator a;
    {
        std::lock_guard<std::mutex> lock(allocator_mu);
        a = allocator_set;
    }
    if (!a.alloc) return fail(SMMO_EINVAL, "dev_buf is NULL and no allocator is set (smmo_set_allocator)");
    void *p = a.alloc(bytes, a.ctx);
    if (!p) return fail(SMMO_ENOMEM, "the allocator returned NULL");
    const smmo_status st = create_heap(s, p, bytes, cfg, stream, out);
    if (st) {
        a.release(p, bytes, a.ctx);
        return st;
    }
    (*out)->owner = a;
    return SMMO_OK;
}

namespace {
smmo_status create_heap(smmo_schema *s, void *dev_buf, size_t bytes, const smmo_config *cfg, smmo_stream stream,
                        smmo_heap **out)
{
    if (!s->nclasses) return fail(SMMO_ESTATE, "schema has no classes");
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return fail(SMMO_EINVAL, "dev_buf must be 256-byte aligned");
    smmo_config c;
    if (cfg) c = *cfg;
    else smmo_config_default(&c);
    if (c.lookup_retries == 0) c.lookup_retries = 1;
    if (c.spin_limit < 1024) c.spin_limit = 1024;
    if (c.block_group != 0 && c.block_group != 1 && c.block_group != 2 && c.block_group != 4)
        return fail(SMMO_EINVAL, "block_group must be 0, 1, 2 or 4");
    if (c.sparse_packing > 2) return fail(SMMO_EINVAL, "sparse_packing must be 0, 1 or 2");
    if (c.streaming_loads > 2) return fail(SMMO_EINVAL, "streaming_loads must be 0, 1 or 2");
    const uint32_t bb = schema_block_bytes(s);
    // largest M whose layout fits
    uint64_t lo = 0, hi = std::min<uint64_t>(bytes / bb, kMaxBlocks);
    Layout L;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        layout_for(s->nclasses, mid, bb, L);
        if (L.total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    if (lo == 0) return fail(SMMO_ENOMEM, "buffer too small for one block");
    const uint64_t M = lo;
    layout_for(s->nclasses, M, bb, L);

    smmo_heap *h = new (std::nothrow) smmo_heap();
    if (!h) return fail(SMMO_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
        h->cu_count = (uint32_t)cus;
    e = hipHostMalloc(reinterpret_cast<void **>(&h->host_ctrl), kCtrlWords * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipHostMalloc");
    }
    char *b = static_cast<char *>(dev_buf);
    HeapView &v = h->v;
    v.ctrl = reinterpret_cast<uint32_t *>(b + L.ctrl);
    v.bm = reinterpret_cast<uint64_t *>(b + L.bm);
    v.type = reinterpret_cast<uint32_t *>(b + L.type);
    v.alloc_bm = reinterpret_cast<uint64_t *>(b + L.alloc);
    v.iter_bm = reinterpret_cast<uint64_t *>(b + L.iter);
    v.R = reinterpret_cast<uint32_t *>(b + L.R);
    v.claim = reinterpret_cast<uint32_t *>(b + L.claim);
    v.blocks = b + L.blocks;
    v.block_bytes = bb;
    v.M = (uint32_t)M;
    v.nclasses = s->nclasses;
    v.nlev = L.nlev;
    v.bm_words = L.bm_words;
    for (uint32_t l = 0; l < kMaxLevels; ++l) {
        v.lvl_off[l] = L.lvl_off[l];
        v.lvl_n[l] = L.lvl_n[l];
    }
    v.retries = c.lookup_retries;
    v.rotation = c.rotation ? 1u : 0u;
    v.coalescing = c.coalescing ? 1u : 0u;
    v.spin_limit = c.spin_limit;
    v.sparse_packing = c.sparse_packing;
    h->schema = s;
    h->base = dev_buf;
    h->bytes = bytes;
    h->cfg = c;
    h->last = static_cast<hipStream_t>(stream);
    const uint64_t work = std::max<uint64_t>(std::max<uint64_t>(M, (1ull + 2ull * s->nclasses) * L.bm_words),
                                             kCtrlWords);
    const uint32_t grid = (uint32_t)std::min<uint64_t>((work + 255) / 256, 16384);
    hipLaunchKernelGGL(k_heap_init, dim3(grid), dim3(256), 0, h->last, v);
    smmo_status st = launch_check("k_heap_init");
    if (st) {
        (void)hipHostFree(h->host_ctrl);
        delete h;
        return st;
    }
    s->frozen = true;
    *out = h;
    return SMMO_OK;
}
} // namespace

smmo_status smmo_heap_free(smmo_heap *h)
{
    if (!h) return SMMO_OK;
    if (h->base) (void)hipStreamSynchronize(h->last);
    if (h->host_ctrl) (void)hipHostFree(h->host_ctrl);
    if (h->base && h->owner.release) h->owner.release(h->base, h->bytes, h->owner.ctx);
    h->base = nullptr;
    delete h;
    return SMMO_OK;
}

smmo_status smmo_parallel_new(smmo_heap *h, uint32_t class_id, uint32_t n, const smmo_field_init *init,
                              uint32_t ninit, uint32_t *out_handles, smmo_stream stream)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    if (class_abstract(h->schema, class_id)) return fail(SMMO_EINVAL, "class is abstract");
    if (ninit && !init) return fail(SMMO_EINVAL, "init is NULL");
    if (n == 0) return SMMO_OK;
    if ((uint64_t)n > 64ull * h->v.M) return fail(SMMO_ENOMEM, "more objects than the heap has slots");
    const smmo_class_info &ci = h->schema->c[class_id];
    if (ninit > ci.nfields) return fail(SMMO_EINVAL, "more initializers than fields");
    FieldSet fs{};
    fs.nf = ci.nfields;
    for (uint32_t j = 0; j < ci.nfields; ++j) {
        const smmo_field_info &fi = ci.f[j];
        fs.f[j] = FieldCopy{fi.offset, fi.stride, fi.size, fi.count, nullptr};
    }
    for (uint32_t k = 0; k < ninit; ++k) {
        if (init[k].field_id >= ci.nfields) return fail(SMMO_EINVAL, "initializer field id out of range");
        if (!init[k].values) return fail(SMMO_EINVAL, "initializer values is NULL");
        if (fs.f[init[k].field_id].src) return fail(SMMO_EINVAL, "field initialized twice");
        fs.f[init[k].field_id].src = init[k].values;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t grid = (uint32_t)(((uint64_t)n + 255) / 256);
    if (h->cfg.bulk_ordered) {
        const uint32_t need = (uint32_t)(((uint64_t)n + 63) / 64);
        hipLaunchKernelGGL(k_bulk_claim, dim3(1), dim3(1024), 0, st, h->v, class_id, need, n % 64);
        if ((s = launch_check("k_bulk_claim"))) return s;
        const uint32_t hgrid = (uint32_t)std::min<uint64_t>((need + 255) / 256, 4096);
        hipLaunchKernelGGL(k_bulk_headers, dim3(hgrid), dim3(256), 0, st, h->v, class_id, need, n % 64);
        if ((s = launch_check("k_bulk_headers"))) return s;
        hipLaunchKernelGGL(k_bulk_init, dim3(grid), dim3(256), 0, st, h->v, fs, n, out_handles);
        if ((s = launch_check("k_bulk_init"))) return s;
    } else {
        hipLaunchKernelGGL(k_new_device, dim3(grid), dim3(256), 0, st, h->v, class_id, fs, n, out_handles);
        if ((s = launch_check("k_new_device"))) return s;
    }
    note_allocation(h, class_id, n, false);
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_parallel_do(smmo_heap *h, uint32_t class_id, uint32_t method_id, const void *args,
                             size_t args_bytes, smmo_stream stream)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    uint32_t nm = 0;
    const MethodEntry *tab = method_table(&nm);
    if (method_id >= nm) return fail(SMMO_EINVAL, "unknown method id");
    const MethodEntry &m = tab[method_id];
    if (args_bytes != m.args_bytes || (m.args_bytes && !args))
        return fail(SMMO_EINVAL, std::string("method '") + m.name + "': wrong argument size");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the class and its descendants: one launch per concrete class, or one
    // for the whole family where the method covers it
    const uint32_t fam = (m.flags & kFamilyLaunch) ? 1u << class_id : class_family(h->schema, class_id);
    // snapshots that smmo_snapshot took of the walked classes are used here,
    // once
    const uint32_t snap = h->snap_pending & class_family(h->schema, class_id);
    h->v.snap = snap;
    for (uint32_t c = 0; c < h->schema->nclasses && !s; ++c) {
        if ((m.flags & kFamilyLaunch) && c == class_id) {
            h->cur_method = method_id;
            s = m.launch(h, c, args, st);
            h->cur_method = 0xFFFFFFFFu;
            continue;
        }
        if (!((fam >> c) & 1) || class_abstract(h->schema, c)) continue;
        h->cur_method = method_id;
        s = m.launch(h, c, args, st);
        h->cur_method = 0xFFFFFFFFu;
    }
    h->v.snap = 0;
    h->snap_pending &= ~snap;
    if (s) return s;
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_snapshot(smmo_heap *h, uint32_t class_id, smmo_stream stream)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t fam = class_family(h->schema, class_id);
    for (uint32_t c = 0; c < h->schema->nclasses; ++c) {
        if (!((fam >> c) & 1) || class_abstract(h->schema, c)) continue;
        // with the packing plan whenever a packed do-all may ask for it
        if ((s = ensure_enumerated(h, c, true, st, h->cfg.sparse_packing != 0, false))) return s;
    }
    h->snap_pending |= fam;
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_set_launch(smmo_heap *h, uint32_t method_id, uint32_t class_id, uint32_t wg_threads,
                            uint32_t grid_waves, uint32_t group)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    uint32_t nm = 0;
    method_table(&nm);
    if (method_id >= nm || method_id >= 64) return fail(SMMO_EINVAL, "unknown method id");
    if (wg_threads != 0 && wg_threads != 64 && wg_threads != 128 && wg_threads != 256 && wg_threads != 512 &&
        wg_threads != 1024)
        return fail(SMMO_EINVAL, "work-group size must be 0 or one of 64, 128, 256, 512, 1024");
    if (group != 0 && group != 1 && group != 2 && group != 4)
        return fail(SMMO_EINVAL, "group must be 0, 1, 2 or 4");
    h->launch_wg[method_id][class_id] = (uint16_t)wg_threads;
    h->launch_group[method_id][class_id] = (uint8_t)group;
    h->launch_waves[method_id][class_id] = grid_waves;
    return SMMO_OK;
}

smmo_status smmo_destroy(smmo_heap *h, uint32_t class_id, const uint32_t *handles, uint32_t n,
                         smmo_stream stream)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    if (n == 0) return SMMO_OK;
    if (!handles) return fail(SMMO_EINVAL, "handles is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    h->snap_pending &= ~(1u << class_id);   // a snapshot would still list the deleted objects
    const uint32_t grid = (uint32_t)(((uint64_t)n + 255) / 256);
    hipLaunchKernelGGL(k_destroy, dim3(grid), dim3(256), 0, st, h->v, class_id, handles, n);
    if ((s = launch_check("k_destroy"))) return s;
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_gather_soa(smmo_heap *h, uint32_t class_id, const uint32_t *field_ids, uint32_t nfields,
                            void *const *out_ptrs, uint32_t *out_handles, uint32_t capacity,
                            uint32_t *out_count, smmo_stream stream)
{
    smmo_status s = check_class(h, class_id);
    if (s) return s;
    if (!out_count) return fail(SMMO_EINVAL, "out_count is NULL");
    if (nfields && (!field_ids || !out_ptrs)) return fail(SMMO_EINVAL, "NULL field list");
    if (nfields > SMMO_MAX_FIELDS) return fail(SMMO_EINVAL, "too many fields");
    for (uint32_t j = 0; j < nfields; ++j)
        if (!out_ptrs[j] && capacity) return fail(SMMO_EINVAL, "output pointer is NULL");
    FieldSet fs{};
    if ((s = build_fieldset(h, class_id, field_ids, nfields, const_cast<const void *const *>(out_ptrs), fs)))
        return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    h->snap_pending &= ~(1u << class_id);
    if ((s = ensure_enumerated(h, class_id, false, st))) return s;
    h->cur_method = 0xFFFFFFFFu;
    const LaunchShape ls = method_shape(h, class_id);
    hipLaunchKernelGGL(k_gather, ls.grid, ls.block, 0, st, h->v, class_id, fs, out_handles, capacity,
                       out_count);
    if ((s = launch_check("k_gather"))) return s;
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_sync(smmo_heap *h)
{
    if (!heap_ok(h)) return fail(SMMO_EINVAL, "heap is NULL or freed");
    smmo_status s = read_ctrl(h, CTRL_ERR, 1);
    if (s) return s;
    return map_device_error(reinterpret_cast<uint32_t *>(h->host_ctrl)[CTRL_ERR]);
}

smmo_status smmo_heap_stats(smmo_heap *h, smmo_stats *out)
{
    if (!heap_ok(h) || !out) return fail(SMMO_EINVAL, "NULL argument");
    smmo_status s = run_stats(h, h->last);
    if (s) return s;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(h->host_ctrl);
    const uint64_t *st = reinterpret_cast<const uint64_t *>(w + CTRL_STATS);
    memset(out, 0, sizeof *out);
    uint64_t slots = 0, used = 0;
    for (uint32_t c = 0; c < h->v.nclasses; ++c) {
        out->live_objects[c] = st[ST_LIVE + c];
        out->blocks[c] = st[ST_BLOCKS + c];
        slots += 64 * st[ST_BLOCKS + c];
        used += st[ST_LIVE + c];
    }
    out->free_blocks = st[ST_FREE];
    out->total_blocks = h->v.M;
    out->fragmentation = slots ? (double)(slots - used) / (double)slots : 0.0;
    out->block_bytes = (uint32_t)h->v.block_bytes;
    for (uint32_t k = 0; k < kEventStripes; ++k) {
        const uint32_t *e = w + CTRL_EVENTS + k * kStripeWords;
        out->slow_paths += *reinterpret_cast<const uint64_t *>(e + EV_SLOW);
        out->alloc_retries += *reinterpret_cast<const uint64_t *>(e + EV_RETRY);
        out->device_news += *reinterpret_cast<const uint64_t *>(e + EV_NEWS);
        out->device_deletes += *reinterpret_cast<const uint64_t *>(e + EV_DELS);
        out->bitmap_spins += *reinterpret_cast<const uint64_t *>(e + EV_SPIN);
        out->lookups += *reinterpret_cast<const uint64_t *>(e + EV_FIND);
    }
    const uint32_t err = w[CTRL_ERR];
    out->device_error = err == 0 ? SMMO_OK : (err == ERR_NOMEM ? SMMO_ENOMEM : SMMO_EDEVICE);
    return SMMO_OK;
}

smmo_status smmo_check_invariants(smmo_heap *h, smmo_invariants *inv)
{
    if (!heap_ok(h) || !inv) return fail(SMMO_EINVAL, "NULL argument");
    smmo_status s = run_stats(h, h->last);
    if (s) return s;
    const uint64_t *st = reinterpret_cast<const uint64_t *>(
        reinterpret_cast<const uint32_t *>(h->host_ctrl) + CTRL_STATS);
    inv->hierarchy_violations = st[ST_HIER];
    inv->state_violations = st[ST_STATE];
    inv->active_violations = st[ST_ACTIVE];
    inv->type_violations = st[ST_TYPE];
    inv->empty_allocated = st[ST_EMPTY];
    return SMMO_OK;
}

smmo_status smmo_clear_error(smmo_heap *h, smmo_stream stream)
{
    if (!heap_ok(h)) return fail(SMMO_EINVAL, "heap is NULL or freed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, h->v.ctrl + CTRL_ERR, 1u);
    smmo_status s = launch_check("k_zero_words");
    if (s) return s;
    h->last = st;
    return SMMO_OK;
}

smmo_status smmo_heap_info(const smmo_heap *h, uint64_t *blocks, uint32_t *block_bytes)
{
    if (!heap_ok(h)) return fail(SMMO_EINVAL, "heap is NULL or freed");
    if (blocks) *blocks = h->v.M;
    if (block_bytes) *block_bytes = (uint32_t)h->v.block_bytes;
    return SMMO_OK;
}

smmo_status smmo_method_id(const char *name, uint32_t *method_id)
{
    if (!name || !method_id) return fail(SMMO_EINVAL, "NULL argument");
    uint32_t n = 0;
    const MethodEntry *t = method_table(&n);
    for (uint32_t i = 0; i < n; ++i)
        if (strcmp(t[i].name, name) == 0) {
            *method_id = i;
            return SMMO_OK;
        }
    return fail(SMMO_EINVAL, std::string("unknown method '") + name + "'");
}

smmo_status smmo_last_error(char *buf, size_t n)
{
    if (!buf || n == 0) return SMMO_EINVAL;
    const size_t k = std::min(n - 1, g_last_error.size());
    memcpy(buf, g_last_error.data(), k);
    buf[k] = 0;
    return SMMO_OK;
}

#ifndef SMMO_SOURCE_HASH
#error "SMMO_SOURCE_HASH is set by the build (paper_1908_05845_amd/build.py)"
#endif
const char *smmo_source_hash(void) { return SMMO_SOURCE_HASH; }

} // extern "C"
