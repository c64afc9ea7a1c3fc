// Memory defragmentation (CompactGpu, Ch.6): blocks of one class that are at
// most n/(n+1) full are merged, each source block into n target blocks, and
// every handle that names a moved object is rewritten through a forwarding
// handle left in the source block.  A pass is four kernels:
//   select   - candidates from the allocation bitmaps (the on-demand variant
//              of the thesis's defrag[T] bitmaps: the allocation and
//              deletion paths keep no extra state)
//   move     - one wavefront per source block copies every field array of
//              its objects into the free slots of its targets, sets the
//              targets' allocation bits with one atomic each, then writes the
//              forwarding handles into the source block and frees it
//   rewrite  - every live HANDLE field of every class, and the caller's
//              external handle arrays; a handle is forwarded iff its block
//              carries the "moved" type mark of this pass
//   finish   - the moved blocks' type mark becomes "no type"
// One wavefront owns a source block and its targets, so the copy and the
// forwarding stores need no second kernel: the wavefront's loads of the
// source block have completed before it overwrites the block's first bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "method_common.hpp"

using namespace smmo;

namespace {

constexpr uint32_t kMoved = 0xFFFFFFFEu;      // type of a source block during its pass
constexpr uint32_t kMaxHandleArrays = 32;     // handle arrays of one class (= SMMO_MAX_FIELDS)

struct MoveK {
    uint32_t cls, B, n, narr;
    uint32_t off[SMMO_MAX_FIELDS];            // every field array of the class
    uint8_t size[SMMO_MAX_FIELDS];            // bytes per element (1 or 4)
};

struct RewriteK {
    uint32_t cls, narr;
    uint32_t off[kMaxHandleArrays];           // the class's HANDLE arrays
};

__global__ void k_defrag_reset(HeapView h, uint32_t all)
{
    if (threadIdx.x == 0) {
        h.ctrl[CTRL_DCOUNT] = 0;
        if (all) {
            h.ctrl[CTRL_DMOVED] = 0;
            h.ctrl[CTRL_DMOVED + 1] = 0;
        }
    }
}

// candidates of class cls (0 < live objects <= cap) appended to D = h.claim
__global__ __launch_bounds__(256) void k_defrag_select(HeapView h, uint32_t cls, uint32_t cap)
{
    if (heap_failed(h)) return;
    const BlockList L = block_list(h, cls);
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t i0 = global_wave_id() * 64; i0 < L.r; i0 += nw * 64) {
        const uint32_t i = i0 + lane;
        bool cand = false;
        uint32_t bid = 0;
        if (i < L.r) {
            bid = L.at(i);
            if (h.type[bid] == cls) {
                const uint32_t c = (uint32_t)__popcll(h.alloc_bm[bid]);
                cand = c > 0 && c <= cap;
            }
        }
        const uint64_t m = __ballot(cand);
        uint32_t base = 0;
        if (lane == 0 && m)
            base = __hip_atomic_fetch_add(h.ctrl + CTRL_DCOUNT, (uint32_t)__popcll(m), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, 0);
        if (cand) h.claim[base + (uint32_t)__popcll(m & ((1ull << lane) - 1))] = bid;
    }
}

// Alg. move_objects and place_forwarding_ptrs in one wavefront per source
// block: source D[w], targets D[w + i B], i = 1..n; the lane holding the
// s-th object of the source takes the s-th free slot of the targets in order.
__global__ __launch_bounds__(256) void k_defrag_move(HeapView h, MoveK p)
{
    const uint32_t w = global_wave_id();
    if (w >= p.B || heap_failed(h)) return;
    const uint32_t lane = lane_id();
    const uint32_t sbid = __builtin_amdgcn_readfirstlane(h.claim[w]);
    const uint64_t sbm = uniform64(h.alloc_bm[sbid]);
    const uint32_t cnt = (uint32_t)__popcll(sbm);
    bool mv = lane < cnt;
    uint32_t tbid = kNoBlock, tslot = 0, ti = 0;
    if (mv) {
        uint32_t t_loc = lane;
        for (uint32_t i = 1; i <= p.n; ++i) {
            const uint32_t tb = h.claim[w + i * p.B];
            const uint64_t fr = ~h.alloc_bm[tb];
            const uint32_t c = (uint32_t)__popcll(fr);
            if (t_loc < c) {
                tbid = tb;
                tslot = nth_set_bit(fr, t_loc);
                ti = i;
                break;
            }
            t_loc -= c;
        }
        if (tbid == kNoBlock) {           // candidates always leave room
            raise_error(h, ERR_INTERNAL);
            mv = false;
        }
    }
    const uint32_t sslot = mv ? nth_set_bit(sbm, lane) : 0;
    if (mv) {
        const char *src = h.block(sbid);
        char *dst = h.block(tbid);
        for (uint32_t a = 0; a < p.narr; ++a) {
            const uint32_t off = p.off[a];
            if (p.size[a] == 1)
                reinterpret_cast<uint8_t *>(dst + off)[tslot] = reinterpret_cast<const uint8_t *>(src + off)[sslot];
            else
                reinterpret_cast<uint32_t *>(dst + off)[tslot] = reinterpret_cast<const uint32_t *>(src + off)[sslot];
        }
    }
    // every load of the source block has been performed before the first
    // 256 bytes of the block are overwritten with forwarding handles
    complete_prior();
    if (mv) reinterpret_cast<uint32_t *>(h.block(sbid))[sslot] = (tbid << 6) | tslot;
    // the targets' new objects; a target that is now full is no longer active
    for (uint32_t i = 1; i <= p.n; ++i) {
        const uint64_t m = wave_or64(mv && ti == i ? 1ull << tslot : 0ull);
        OpQueue q;
        q.reset();
        if (m && lane == 0) {
            const uint32_t tb = h.claim[w + i * p.B];
            const uint64_t prev = aor(h.alloc_bm + tb, m);
            if ((prev | m) == ~0ull) q.push(bm_active(p.cls), tb, -1);
        }
        run_ops_wave(h, q);
    }
    // the source is empty: invalidated, marked as moved, and free
    OpQueue q;
    q.reset();
    if (lane == 0) {
        __hip_atomic_store(h.alloc_bm + sbid, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(h.type + sbid, kMoved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        complete_prior();
        q.push(bm_active(p.cls), sbid, -1);
        q.push(bm_alloc(p.cls), sbid, -1);
        q.push(BM_FREE, sbid, +1);
        __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(h.ctrl + CTRL_DMOVED),
                               (unsigned long long)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    run_ops_wave(h, q);
}

// Alg. rewrite_pointer on one handle value
__device__ __forceinline__ uint32_t forwarded(const HeapView &h, uint32_t hd)
{
    if (hd == kNull) return hd;
    const uint32_t hb = (hd & 0x7FFFFFFFu) >> 6;
    if (hb >= h.M || h.type[hb] != kMoved) return hd;
    return reinterpret_cast<const uint32_t *>(h.block(hb))[hd & 63] | (hd & 0x80000000u);
}

__global__ __launch_bounds__(1024) void k_defrag_rewrite(HeapView h, RewriteK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        for (uint32_t a = 0; a < p.narr; ++a) {
            uint32_t &v = farr<uint32_t>(h, bid, p.off[a])[s];
            const uint32_t hd = v;
            const uint32_t nv = forwarded(h, hd);
            if (nv != hd) v = nv;
        }
    });
}

__global__ __launch_bounds__(256) void k_defrag_rewrite_ext(HeapView h, uint32_t *a, uint64_t n)
{
    if (heap_failed(h)) return;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t hd = a[i];
        const uint32_t nv = forwarded(h, hd);
        if (nv != hd) a[i] = nv;
    }
}

__global__ __launch_bounds__(256) void k_defrag_finish(HeapView h, uint32_t B)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) h.type[h.claim[i]] = kNull;
}

} // namespace

smmo_status smmo_defragment(smmo_heap *h, uint32_t class_id, uint32_t n, uint32_t k1, uint32_t max_passes,
                            const smmo_handle_array *ext, uint32_t next, smmo_stream stream,
                            uint32_t *out_passes, uint64_t *out_moved)
{
    smmo_status s = heap_check_class(h, class_id);
    if (s) return s;
    if (n < 1 || n > 8) return fail(SMMO_EINVAL, "defragment: n must be 1..8");
    if (next && !ext) return fail(SMMO_EINVAL, "defragment: external array list is NULL");
    for (uint32_t e = 0; e < next; ++e)
        if (!ext[e].handles && ext[e].count) return fail(SMMO_EINVAL, "defragment: external array is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const smmo_schema &sc = *h->schema;
    MoveK mk{};
    mk.cls = class_id;
    mk.n = n;
    const smmo_class_info &ci = sc.c[class_id];
    for (uint32_t f = 0; f < ci.nfields; ++f)
        for (uint32_t q = 0; q < ci.f[f].count; ++q) {
            mk.off[mk.narr] = ci.f[f].offset + q * ci.f[f].stride;
            mk.size[mk.narr] = (uint8_t)ci.f[f].size;
            mk.narr++;
        }
    RewriteK rk[SMMO_MAX_CLASSES];
    uint32_t nrk = 0;
    for (uint32_t c = 0; c < sc.nclasses; ++c) {
        RewriteK k{};
        k.cls = c;
        for (uint32_t f = 0; f < sc.c[c].nfields; ++f)
            if (sc.c[c].f[f].dtype == SMMO_HANDLE)
                for (uint32_t q = 0; q < sc.c[c].f[f].count; ++q) k.off[k.narr++] = sc.c[c].f[f].offset + q * sc.c[c].f[f].stride;
        if (k.narr) rk[nrk++] = k;
    }
    const uint32_t cap = 64 * n / (n + 1);
    hipLaunchKernelGGL(k_defrag_reset, dim3(1), dim3(64), 0, st, h->v, 1u);
    if ((s = heap_launch_check("k_defrag_reset"))) return s;
    h->last = st;
    h->snap_pending &= ~(1u << class_id);   // its objects move: a snapshot of the class no longer holds
    uint32_t passes = 0;
    while (passes < max_passes) {
        if ((s = ensure_enumerated(h, class_id, false, st))) return s;
        hipLaunchKernelGGL(k_defrag_reset, dim3(1), dim3(64), 0, st, h->v, 0u);
        const uint64_t blocks = std::max<uint64_t>(1, h->ub_blocks[class_id]);
        const uint32_t sgrid = (uint32_t)std::min<uint64_t>((blocks + 255) / 256, 4096);
        hipLaunchKernelGGL(k_defrag_select, dim3(sgrid), dim3(256), 0, st, h->v, class_id, cap);
        if ((s = heap_launch_check("k_defrag_select"))) return s;
        h->last = st;
        if ((s = heap_read_ctrl(h, CTRL_DCOUNT, 1))) return s;
        const uint32_t d = reinterpret_cast<const uint32_t *>(h->host_ctrl)[CTRL_DCOUNT];
        if (d <= k1 || d < n + 1) break;
        mk.B = d / (n + 1);
        hipLaunchKernelGGL(k_defrag_move, dim3((mk.B + 3) / 4), dim3(256), 0, st, h->v, mk);
        if ((s = heap_launch_check("k_defrag_move"))) return s;
        h->rstate[class_id] = R_DIRTY;
        for (uint32_t i = 0; i < nrk; ++i) {
            if ((s = ensure_enumerated(h, rk[i].cls, false, st))) return s;
            const LaunchShape ls = method_shape(h, rk[i].cls);
            hipLaunchKernelGGL(k_defrag_rewrite, ls.grid, ls.block, 0, st, h->v, rk[i]);
            if ((s = heap_launch_check("k_defrag_rewrite"))) return s;
        }
        for (uint32_t e = 0; e < next; ++e) {
            if (!ext[e].count) continue;
            const uint32_t g = (uint32_t)std::min<uint64_t>((ext[e].count + 255) / 256, 4096);
            hipLaunchKernelGGL(k_defrag_rewrite_ext, dim3(g), dim3(256), 0, st, h->v, ext[e].handles, ext[e].count);
            if ((s = heap_launch_check("k_defrag_rewrite_ext"))) return s;
        }
        hipLaunchKernelGGL(k_defrag_finish, dim3((mk.B + 255) / 256), dim3(256), 0, st, h->v, mk.B);
        if ((s = heap_launch_check("k_defrag_finish"))) return s;
        ++passes;
    }
    h->last = st;
    if ((s = heap_read_ctrl(h, CTRL_DMOVED, 2))) return s;
    if (out_passes) *out_passes = passes;
    if (out_moved)
        *out_moved = *reinterpret_cast<const uint64_t *>(reinterpret_cast<const uint32_t *>(h->host_ctrl) + CTRL_DMOVED);
    return smmo_sync(h);
}
