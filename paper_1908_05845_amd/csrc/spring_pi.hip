// Spring-mass methods for a node adjacency that is partly inlined (Ch.4
// sec.4.3.1 "SOA with Partial Inlining"): the first K slots are SOA arrays in
// the node's block, the others an array outside the heap indexed from a
// per-node offset (field contracts in include/smmo_methods.h).  The force law
// and the break decision are those of the spring kernels; a low-degree node
// touches only its inline slots, a hub reads its other slots as gathers.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

using namespace smmo;

namespace {

constexpr uint32_t kB = 0x80000000u;      // slot tag: this node is the spring's endpoint b

struct PiK {
    uint32_t node_cls, spring_cls;
    uint32_t s_a, s_b, s_k, s_L0, s_fx, s_fy, s_sa, s_sb;                  // Spring fields
    uint32_t n_x, n_y, n_vx, n_vy, n_m, n_adj, n_adj_stride, n_more, n_cap; // Node fields
    uint32_t K;                                                           // inlined slots
    float dt, limit;
    uint32_t *ovf;
    uint64_t ovf_len;
    uint32_t wpg;             // wavefronts per work-group of this launch
};

// slot q of node `node`, or nullptr (and the device error set) if q is not a
// slot of the node or its overflow index is outside the array
__device__ __forceinline__ uint32_t *slot_ptr(const HeapView &h, const PiK &p, uint32_t node, uint32_t q)
{
    const int32_t cap = fref<int32_t>(h, node, p.n_cap);
    if ((int32_t)q >= cap) {
        raise_error(h, ERR_BADHANDLE);
        return nullptr;
    }
    if (q < p.K) return &fref<uint32_t>(h, node, p.n_adj + q * p.n_adj_stride);
    const int64_t idx = (int64_t)fref<int32_t>(h, node, p.n_more) + (int64_t)(q - p.K);
    if (idx < 0 || (uint64_t)idx >= p.ovf_len) {
        raise_error(h, ERR_BADHANDLE);
        return nullptr;
    }
    return p.ovf + idx;
}

__device__ __forceinline__ bool pi_valid(const HeapView &h, uint32_t handle)
{
    if ((handle >> 6) < h.M) return true;
    raise_error(h, ERR_BADHANDLE);
    return false;
}

// Spring::compute_force with the strain break (the spring kernels' float32
// operation order, no contraction)
__global__ __launch_bounds__(1024) void k_pi_force(HeapView h, PiK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<1>(h, p.spring_cls, p.wpg, [&](const BlockHeads<1> &hd) {
#pragma clang fp contract(off)
        const uint32_t bid = hd.bid[0];
        // the spring's own fields for all 64 slots at once, with its handles,
        // issued before the header is used
        uint32_t a = farr<uint32_t>(h, bid, p.s_a)[s];
        uint32_t b = farr<uint32_t>(h, bid, p.s_b)[s];
        const float L0 = farr<float>(h, bid, p.s_L0)[s], k = farr<float>(h, bid, p.s_k)[s];
        if (!hd.own(0)) return;   // (uniform over the wavefront; stores below are full-width)
        bool live = (hd.bm(0) >> s) & 1;
        if (live) live = pi_valid(h, a) && pi_valid(h, b);
        if (!live) a = b = 0;
        float fx = 0.f, fy = 0.f;
        bool brk = false;
        if (live) {
            const float dx = fref<float>(h, b, p.n_x) - fref<float>(h, a, p.n_x);
            const float dy = fref<float>(h, b, p.n_y) - fref<float>(h, a, p.n_y);
            const float dy2 = dy * dy;
            const float l = __builtin_sqrtf(__builtin_fmaf(dx, dx, dy2));
            brk = (l - L0) / L0 > p.limit;
            if (!brk) {
                const float c = k * (l - L0) / l;
                fx = c * dx;
                fy = c * dy;
            }
        }
        farr<float>(h, bid, p.s_fx)[s] = fx;
        farr<float>(h, bid, p.s_fy)[s] = fy;
        if (brk) {
            uint32_t *qa = slot_ptr(h, p, a, farr<uint8_t>(h, bid, p.s_sa)[s]);
            uint32_t *qb = slot_ptr(h, p, b, farr<uint8_t>(h, bid, p.s_sb)[s]);
            if (qa) *qa = kNull;
            if (qb) *qb = kNull;
        }
        wave_release_own_block(h, p.spring_cls, bid, __ballot(brk));
    });
}

// the signed force of the spring in slot entry e (0 for an empty slot)
__device__ __forceinline__ void add_slot(const HeapView &h, const PiK &p, uint32_t e, float &Fx, float &Fy)
{
    if (e == kNull) return;
    const uint32_t sp = e & ~kB;
    if (!pi_valid(h, sp)) return;
    const float fx = fref<float>(h, sp, p.s_fx), fy = fref<float>(h, sp, p.s_fy);
    Fx += (e & kB) ? -fx : fx;
    Fy += (e & kB) ? -fy : fy;
}

// sum over the 64 lanes in a fixed order (butterfly)
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// a node with more out-of-line slots than this is summed by the whole
// wavefront (the thesis's nested parallelism for high-degree vertices)
constexpr int32_t kLaneSerialSlots = 8;

// Node::update: the attached springs' forces (inline slots, then the node's
// out-of-line slots), then v and x.  Out-of-line slots of a hub are gathered
// by all lanes of the wavefront, 64 at a time, and summed with a wavefront
// reduction, instead of one lane walking them while the others wait.
__global__ __launch_bounds__(1024) void k_pi_node(HeapView h, PiK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<1>(h, p.node_cls, p.wpg, [&](const BlockHeads<1> &hd) {
        const uint32_t bid = hd.bid[0];
        // the slot count and overflow index, issued before the header is used
        const int32_t cap0 = farr<int32_t>(h, bid, p.n_cap)[s];
        const int32_t more0 = farr<int32_t>(h, bid, p.n_more)[s];
        const bool live = (hd.bm(0) >> s) & 1;
        const int32_t cap = live ? cap0 : 0;
        const int64_t base = live ? more0 : 0;
        const int32_t extra = cap - (int32_t)p.K;
        float Fx = 0.f, Fy = 0.f;
        if (live) {
            for (uint32_t q = 0; q < p.K; ++q) {           // wave-uniform trip count
                if ((int32_t)q >= cap) break;
                add_slot(h, p, farr<uint32_t>(h, bid, p.n_adj + q * p.n_adj_stride)[s], Fx, Fy);
            }
            if (extra > 0 && extra <= kLaneSerialSlots) {
                if (base < 0 || (uint64_t)(base + extra) > p.ovf_len) raise_error(h, ERR_BADHANDLE);
                else
                    for (int32_t q = 0; q < extra; ++q) add_slot(h, p, p.ovf[base + q], Fx, Fy);
            }
        }
        // hubs: the wavefront takes them one at a time
        uint64_t hubs = __ballot(live && extra > kLaneSerialSlots);
        while (hubs) {
            const uint32_t j = (uint32_t)(__ffsll((unsigned long long)hubs) - 1);
            hubs &= hubs - 1;
            const int32_t ej = __shfl(extra, (int)j);
            const int64_t bj = (int64_t)__shfl((int)base, (int)j);
            float sx = 0.f, sy = 0.f;
            if (bj >= 0 && (uint64_t)(bj + ej) <= p.ovf_len) {
                for (int32_t q = (int32_t)s; q < ej; q += 64) add_slot(h, p, p.ovf[bj + q], sx, sy);
            } else if (s == j) {
                raise_error(h, ERR_BADHANDLE);
            }
            sx = wave_sum(sx);
            sy = wave_sum(sy);
            if (s == j) {
                Fx += sx;
                Fy += sy;
            }
        }
        if (!live) return;
        const float m = farr<float>(h, bid, p.n_m)[s];
        float &vx = farr<float>(h, bid, p.n_vx)[s];
        float &vy = farr<float>(h, bid, p.n_vy)[s];
        vx += Fx / m * p.dt;
        vy += Fy / m * p.dt;
        farr<float>(h, bid, p.n_x)[s] += vx * p.dt;
        farr<float>(h, bid, p.n_y)[s] += vy * p.dt;
    });
}

// Spring::link: register the spring in its endpoints' slots
__global__ __launch_bounds__(1024) void k_pi_link(HeapView h, PiK p)
{
    for_each_block(h, p.spring_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t a = farr<uint32_t>(h, bid, p.s_a)[s], b = farr<uint32_t>(h, bid, p.s_b)[s];
        if (!pi_valid(h, a) || !pi_valid(h, b)) return;
        const uint32_t me = (bid << 6) | s;
        uint32_t *qa = slot_ptr(h, p, a, farr<uint8_t>(h, bid, p.s_sa)[s]);
        uint32_t *qb = slot_ptr(h, p, b, farr<uint8_t>(h, bid, p.s_sb)[s]);
        if (qa) *qa = me;
        if (qb) *qb = me | kB;
    });
}

smmo_status bind_spring_pi(smmo_heap *h, const smmo_spring_pi_args &a, PiK &k)
{
    const smmo_schema *sc = h->schema;
    if (a.node_class >= sc->nclasses || a.spring_class >= sc->nclasses || a.node_class == a.spring_class)
        return fail(SMMO_EINVAL, "spring_pi: bad class ids");
    if (!(a.dt == a.dt) || !(a.strain_limit == a.strain_limit)) return fail(SMMO_EINVAL, "spring_pi: NaN parameter");
    if (!a.overflow && a.overflow_len) return fail(SMMO_EINVAL, "spring_pi: overflow is NULL");
    memset(&k, 0, sizeof k);
    k.node_cls = a.node_class;
    k.spring_cls = a.spring_class;
    BIND(a.spring_class, "a", SMMO_HANDLE, 1, &k.s_a, nullptr);
    BIND(a.spring_class, "b", SMMO_HANDLE, 1, &k.s_b, nullptr);
    BIND(a.spring_class, "k", SMMO_F32, 1, &k.s_k, nullptr);
    BIND(a.spring_class, "L0", SMMO_F32, 1, &k.s_L0, nullptr);
    BIND(a.spring_class, "fx", SMMO_F32, 1, &k.s_fx, nullptr);
    BIND(a.spring_class, "fy", SMMO_F32, 1, &k.s_fy, nullptr);
    BIND(a.spring_class, "slot_a", SMMO_U8, 1, &k.s_sa, nullptr);
    BIND(a.spring_class, "slot_b", SMMO_U8, 1, &k.s_sb, nullptr);
    BIND(a.node_class, "x", SMMO_F32, 1, &k.n_x, nullptr);
    BIND(a.node_class, "y", SMMO_F32, 1, &k.n_y, nullptr);
    BIND(a.node_class, "vx", SMMO_F32, 1, &k.n_vx, nullptr);
    BIND(a.node_class, "vy", SMMO_F32, 1, &k.n_vy, nullptr);
    BIND(a.node_class, "m", SMMO_F32, 1, &k.n_m, nullptr);
    BIND(a.node_class, "adj", SMMO_HANDLE, 0, &k.n_adj, &k.n_adj_stride);
    BIND(a.node_class, "more", SMMO_I32, 1, &k.n_more, nullptr);
    BIND(a.node_class, "cap", SMMO_I32, 1, &k.n_cap, nullptr);
    const smmo_class_info &ci = sc->c[a.node_class];
    for (uint32_t j = 0; j < ci.nfields; ++j)
        if (strcmp(ci.f[j].name, "adj") == 0) k.K = ci.f[j].count;
    k.dt = a.dt;
    k.limit = a.strain_limit;
    k.ovf = a.overflow;
    k.ovf_len = a.overflow_len;
    return SMMO_OK;
}

// Which: 0 force, 1 node_update, 2 link
template <int Which>
smmo_status launch_spring_pi(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_spring_pi_args a;
    memcpy(&a, args, sizeof a);
    PiK k;
    smmo_status s = cached_bind(h, (const void *)&launch_spring_pi<0>, cls, a, k,
                                [&] { return bind_spring_pi(h, a, k); });
    if (s) return s;
    const uint32_t want = Which == 1 ? a.node_class : a.spring_class;
    if (cls != want) return fail(SMMO_EINVAL, "spring_pi: method runs on a different class");
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    const LaunchShape ls = method_shape(h, cls);
    k.wpg = ls.block.x / 64;
    if (Which == 0) hipLaunchKernelGGL(k_pi_force, ls.grid, ls.block, 0, st, h->v, k);
    if (Which == 1) hipLaunchKernelGGL(k_pi_node, ls.grid, ls.block, 0, st, h->v, k);
    if (Which == 2) hipLaunchKernelGGL(k_pi_link, ls.grid, ls.block, 0, st, h->v, k);
    return launched("spring_pi kernel");
}

} // namespace

namespace smmo {
smmo_status launch_spring_pi_force(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring_pi<0>(h, c, a, s); }
smmo_status launch_spring_pi_node_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring_pi<1>(h, c, a, s); }
smmo_status launch_spring_pi_link(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring_pi<2>(h, c, a, s); }
} // namespace smmo
