// Spring-mass methods (thesis Ch.7 "structure", its compute steps):
// Spring::force, Node::update and the topology link; field contracts in
// include/smmo_methods.h.  These are the kernels of the spring step; the
// launch conventions are those of every method kernel (method_common.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

using namespace smmo;

namespace {

// ======================================================== spring-mass =====
struct SpringK {
    uint32_t node_cls, spring_cls;
    uint32_t s_a, s_b, s_k, s_L0, s_fx, s_fy, s_sa, s_sb;      // Spring fields
    uint32_t n_x, n_y, n_vx, n_vy, n_m, n_adj, n_adj_stride;   // Node fields
    float dt, limit;
    uint32_t tension_only;
    uint32_t wpg;             // wavefronts per work-group of this launch
};

// A load of a field that a do-all reads once per object (not one of the
// gathered fields): with NT it carries the non-temporal hint, so that these
// lines do not displace the gathered ones (node positions, spring forces,
// each read by several objects) from the L2 and the MALL.
template <bool NT, class T>
__device__ __forceinline__ T stream_ld(const T &r)
{
    if constexpr (NT) return __builtin_nontemporal_load(&r);
    else return r;
}

// The break decision is integer-valued, so it is evaluated in float32 with a
// fixed operation order (no contraction): dx, dy; l2 = fma(dx, dx, dy*dy);
// l = sqrt(l2) (correctly rounded); strain = (l - L0) / L0 (correctly rounded).
__device__ __forceinline__ bool spring_breaks(float dx, float dy, float L0, float limit, float &l)
{
#pragma clang fp contract(off)
    const float dy2 = dy * dy;
    const float l2 = __builtin_fmaf(dx, dx, dy2);
    l = __builtin_sqrtf(l2);
    const float strain = (l - L0) / L0;
    return strain > limit;
}

// Spring::compute_force (Ch.7 "structure"): Hooke's law on the length change;
// a spring strained past the limit empties its two adjacency slots and
// deletes itself (the thesis's remove_spring followed by destroy).  A
// wavefront works on U blocks at once: the spring fields of all U blocks are
// loaded, then all position gathers issued, then the forces computed.
template <int U, bool NT>
__device__ __forceinline__ void spring_force(const HeapView &h, const SpringK &p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<U>(h, p.spring_cls, p.wpg, [&](const BlockHeads<U> &hd) {
        const uint32_t *bid = hd.bid;
        uint32_t a[U], b[U];
        float k[U], L0[U], xa[U], ya[U], xb[U], yb[U];
        bool live[U], own[U];
        // the blocks' own fields for all 64 slots (one contiguous run each),
        // issued before the headers are used
#pragma unroll
        for (int j = 0; j < U; ++j) {
            a[j] = stream_ld<NT>(farr<uint32_t>(h, bid[j], p.s_a)[s]);
            b[j] = stream_ld<NT>(farr<uint32_t>(h, bid[j], p.s_b)[s]);
            k[j] = stream_ld<NT>(farr<float>(h, bid[j], p.s_k)[s]);
            L0[j] = stream_ld<NT>(farr<float>(h, bid[j], p.s_L0)[s]);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            own[j] = hd.own(j);
            live[j] = (hd.bm(j) >> s) & 1;
        }
        // gathers through the node handles, live slots only
#pragma unroll
        for (int j = 0; j < U; ++j) {
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
            if (!own[j]) continue;
            const float dx = xb[j] - xa[j], dy = yb[j] - ya[j];
            float l;
            const bool brk = live[j] && spring_breaks(dx, dy, L0[j], p.limit, l);
            float fx = 0.f, fy = 0.f;
            if (live[j] && !brk && (!p.tension_only || l > L0[j])) {
                const float c = k[j] * (l - L0[j]) / l;
                fx = c * dx;
                fy = c * dy;
            }
            // full-width stores: dead and broken slots get 0, never read
            farr<float>(h, bid[j], p.s_fx)[s] = fx;
            farr<float>(h, bid[j], p.s_fy)[s] = fy;
            if (brk) {
                const uint32_t qa = farr<uint8_t>(h, bid[j], p.s_sa)[s];
                const uint32_t qb = farr<uint8_t>(h, bid[j], p.s_sb)[s];
                fref<uint32_t>(h, a[j], p.n_adj + qa * p.n_adj_stride) = kNull;
                fref<uint32_t>(h, b[j], p.n_adj + qb * p.n_adj_stride) = kNull;
            }
            wave_release_own_block(h, p.spring_cls, bid[j], __ballot(brk));
        }
    });
}

// One and two blocks per iteration: the registers are held to what eight
// wavefronts per SIMD allow (the rare release path of a breaking spring would
// otherwise raise the scalar registers past that), so one grid of 32
// wavefronts per CU stays resident.  Four blocks per iteration need more
// registers than that and keep the compiler's allocation.
template <int U, bool NT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spring_force(HeapView h,
                                                                                                 SpringK p)
{
    spring_force<U, NT>(h, p);
}

template <bool NT>
__global__ __launch_bounds__(1024) void k_spring_force4(HeapView h, SpringK p)
{
    spring_force<4, NT>(h, p);
}

// Node::update: sum the attached springs' forces in slot order (+f if this
// node is endpoint a, -f if b), then v += F/m dt, x += v dt.  U blocks at
// once, as in the force kernel.
template <int U, bool NT>
__global__ __launch_bounds__(1024) void k_spring_node(HeapView h, SpringK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<U>(h, p.node_cls, p.wpg, [&](const BlockHeads<U> &hd) {
        const uint32_t *bid = hd.bid;
        uint32_t e[U][8];
        float m[U], x[U], y[U], vx[U], vy[U], Fx[U], Fy[U];
        bool live[U];
        // the blocks' fields, issued before the headers are used
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                e[j][q] = stream_ld<NT>(farr<uint32_t>(h, bid[j], p.n_adj + q * p.n_adj_stride)[s]);
            m[j] = stream_ld<NT>(farr<float>(h, bid[j], p.n_m)[s]);
            x[j] = stream_ld<NT>(farr<float>(h, bid[j], p.n_x)[s]);
            y[j] = stream_ld<NT>(farr<float>(h, bid[j], p.n_y)[s]);
            vx[j] = stream_ld<NT>(farr<float>(h, bid[j], p.n_vx)[s]);
            vy[j] = stream_ld<NT>(farr<float>(h, bid[j], p.n_vy)[s]);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) live[j] = (hd.bm(j) >> s) & 1;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            float gx[8], gy[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                gx[q] = 0.f;
                gy[q] = 0.f;
                if (live[j] && e[j][q] != kNull) {
                    const uint32_t sh = e[j][q] & 0x7FFFFFFFu;
                    gx[q] = fref<float>(h, sh, p.s_fx);
                    gy[q] = fref<float>(h, sh, p.s_fy);
                }
            }
            Fx[j] = 0.f;
            Fy[j] = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (e[j][q] == kNull) continue;
                if (e[j][q] >> 31) {
                    Fx[j] -= gx[q];
                    Fy[j] -= gy[q];
                } else {
                    Fx[j] += gx[q];
                    Fy[j] += gy[q];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!live[j]) continue;
            vx[j] += Fx[j] / m[j] * p.dt;
            vy[j] += Fy[j] / m[j] * p.dt;
            x[j] += vx[j] * p.dt;
            y[j] += vy[j] * p.dt;
            farr<float>(h, bid[j], p.n_vx)[s] = vx[j];
            farr<float>(h, bid[j], p.n_vy)[s] = vy[j];
            farr<float>(h, bid[j], p.n_x)[s] = x[j];
            farr<float>(h, bid[j], p.n_y)[s] = y[j];
        }
    });
}

// Spring::link: registers the spring in its two nodes' adjacency slots
// (slot_a of a, slot_b of b, the latter flagged as endpoint b).  Builds a
// mesh's topology on the device after parallel_new of nodes and springs;
// every (node, slot) pair belongs to one spring, so the writes never collide.
__global__ __launch_bounds__(1024) void k_spring_link(HeapView h, SpringK p)
{
    for_each_block(h, p.spring_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t self = (bid << 6) | s;
        const uint32_t a = farr<uint32_t>(h, bid, p.s_a)[s];
        const uint32_t b = farr<uint32_t>(h, bid, p.s_b)[s];
        const uint32_t qa = farr<uint8_t>(h, bid, p.s_sa)[s];
        const uint32_t qb = farr<uint8_t>(h, bid, p.s_sb)[s];
        if (qa >= 8 || qb >= 8) {
            raise_error(h, ERR_BADHANDLE);
            return;
        }
        fref<uint32_t>(h, a, p.n_adj + qa * p.n_adj_stride) = self;
        fref<uint32_t>(h, b, p.n_adj + qb * p.n_adj_stride) = self | 0x80000000u;
    });
}

smmo_status bind_spring(smmo_heap *h, const smmo_spring_args &a, SpringK &k)
{
    const uint32_t nc = h->schema->nclasses;
    if (a.node_class >= nc || a.spring_class >= nc || a.node_class == a.spring_class)
        return fail(SMMO_EINVAL, "spring: bad class ids");
    if (!(a.dt == a.dt) || !(a.strain_limit == a.strain_limit)) return fail(SMMO_EINVAL, "spring: NaN parameter");
    if (a.flags & ~SMMO_SPRING_TENSION_ONLY) return fail(SMMO_EINVAL, "spring: unknown flags");
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
    BIND(a.node_class, "adj", SMMO_HANDLE, 8, &k.n_adj, &k.n_adj_stride);
    k.dt = a.dt;
    k.limit = a.strain_limit;
    k.tension_only = (a.flags & SMMO_SPRING_TENSION_ONLY) ? 1u : 0u;
    return SMMO_OK;
}

// blocks per wavefront iteration of the spring do-alls unless set otherwise
constexpr uint32_t kSpringGroup = 1;

// the MALL (Infinity Cache) of an MI355X, in front of HBM
constexpr uint64_t kMallBytes = 256ull << 20;

// whether the step's once-read fields get the non-temporal hint (the heap's
// streaming_loads; automatic: when the node and spring blocks exceed the
// MALL, so that a step's blocks cannot stay in it for the next step anyway)
bool streaming(const smmo_heap *h, const SpringK &k)
{
    if (h->cfg.streaming_loads) return h->cfg.streaming_loads == 2;
    return (h->ub_blocks[k.node_cls] + h->ub_blocks[k.spring_cls]) * (uint64_t)h->v.block_bytes > kMallBytes;
}

template <int U, bool NT>
void launch_force(const LaunchShape &ls, hipStream_t st, const HeapView &v, const SpringK &k)
{
    if constexpr (U == 4) hipLaunchKernelGGL(k_spring_force4<NT>, ls.grid, ls.block, 0, st, v, k);
    else hipLaunchKernelGGL((k_spring_force<U, NT>), ls.grid, ls.block, 0, st, v, k);
}

template <int Which>
smmo_status launch_spring(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_spring_args a;
    memcpy(&a, args, sizeof a);
    SpringK k;
    smmo_status s = cached_bind(h, (const void *)&launch_spring<Which>, cls, a, k,
                                [&] { return bind_spring(h, a, k); });
    if (s) return s;
    if (cls != (Which == 1 ? a.node_class : a.spring_class))
        return fail(SMMO_EINVAL, "spring: method runs on a different class");
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    const LaunchShape ls = method_shape(h, cls, kSpringGroup);
    k.wpg = ls.block.x / 64;
    const bool nt = Which != 2 && streaming(h, k);
    if (Which == 0) {
        if (ls.group == 4) nt ? launch_force<4, true>(ls, st, h->v, k) : launch_force<4, false>(ls, st, h->v, k);
        else if (ls.group == 2) nt ? launch_force<2, true>(ls, st, h->v, k) : launch_force<2, false>(ls, st, h->v, k);
        else nt ? launch_force<1, true>(ls, st, h->v, k) : launch_force<1, false>(ls, st, h->v, k);
    }
    if (Which == 1) {
        if (ls.group == 4) {
            if (nt) hipLaunchKernelGGL((k_spring_node<4, true>), ls.grid, ls.block, 0, st, h->v, k);
            else hipLaunchKernelGGL((k_spring_node<4, false>), ls.grid, ls.block, 0, st, h->v, k);
        } else if (ls.group == 2) {
            if (nt) hipLaunchKernelGGL((k_spring_node<2, true>), ls.grid, ls.block, 0, st, h->v, k);
            else hipLaunchKernelGGL((k_spring_node<2, false>), ls.grid, ls.block, 0, st, h->v, k);
        } else {
            if (nt) hipLaunchKernelGGL((k_spring_node<1, true>), ls.grid, ls.block, 0, st, h->v, k);
            else hipLaunchKernelGGL((k_spring_node<1, false>), ls.grid, ls.block, 0, st, h->v, k);
        }
    }
    if (Which == 2) {
        const LaunchShape l1 = method_shape(h, cls);
        hipLaunchKernelGGL(k_spring_link, l1.grid, l1.block, 0, st, h->v, k);
    }
    return launched("spring kernel");
}

} // namespace

namespace smmo {
smmo_status launch_spring_force(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring<0>(h, c, a, s); }
smmo_status launch_spring_node_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring<1>(h, c, a, s); }
smmo_status launch_spring_link(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spring<2>(h, c, a, s); }
} // namespace smmo
