// Reverse mode through the spring-mesh step (methods "adjoint.*", contracts
// in include/smmo_methods.h).  Each reverse step is a Node pass and a Spring
// pass, like the forward step: the Node pass first adds the previous Spring
// pass's terms (in adjacency-slot order, no atomics) and then forms
// mu = lv + dt lx and w = M^-1 mu; the Spring pass turns w into the terms
// dt K g of both endpoints and accumulates dL/dk.  Positions of step n come
// from a tape of planes indexed by node handle, filled by "adjoint.step_node"
// (or "adjoint.record") while a segment is recomputed from an (x, v)
// checkpoint ("adjoint.save" / "adjoint.load").
#include <hip/hip_runtime.h>

#include <cstring>

#include "method_common.hpp"

using namespace smmo;

namespace {

struct AdjK {
    uint32_t node_cls, spring_cls;
    uint32_t n_x, n_y, n_vx, n_vy, n_m, n_adj, n_adj_stride, n_id;
    uint32_t n_lx, n_ly, n_lvx, n_lvy, n_wx, n_wy;
    uint32_t s_a, s_b, s_k, s_L0, s_cx, s_cy, s_gk, s_fx, s_fy;
    float dt;
    uint32_t mode;
    float *tape;
    uint64_t plane;
    uint32_t slot;
    uint32_t seed_count;
    const float *seed_x, *seed_y, *seed_vx, *seed_vy;
    uint32_t wpg;             // wavefronts per work-group of this launch
};

struct AdjKey {
    uint32_t node_class, spring_class;
};

__device__ __forceinline__ float *plane_ptr(const AdjK &p, uint32_t plane_index)
{
    return p.tape + (uint64_t)plane_index * p.plane;
}

__global__ __launch_bounds__(1024) void k_adj_record(HeapView h, AdjK p)
{
    if (heap_failed(h)) return;
    float *px = plane_ptr(p, 2 * p.slot), *py = plane_ptr(p, 2 * p.slot + 1);
    for_each_block(h, p.node_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t hd = (bid << 6) | s;
        px[hd] = farr<float>(h, bid, p.n_x)[s];
        py[hd] = farr<float>(h, bid, p.n_y)[s];
    });
}

// Node pass of the forward step (the update of "spring.node_update": the
// springs' forces summed in slot order, then symplectic Euler), which with a
// tape also stores the new positions in tape plane pair `slot`, so that a
// recomputed segment fills its tape without launches of its own.  The
// adjoint's forward run takes the same kernel without a tape: the recomputed
// positions are those of the forward run bit for bit.
template <int U>
__global__ __launch_bounds__(1024) void k_adj_step_node(HeapView h, AdjK p)
{
    const uint32_t s = lane_id();
    float *px = p.tape ? plane_ptr(p, 2 * p.slot) : nullptr;
    float *py = p.tape ? plane_ptr(p, 2 * p.slot + 1) : nullptr;
    for_each_block_heads<U>(h, p.node_cls, p.wpg, [&](const BlockHeads<U> &hd) {
        const uint32_t *bid = hd.bid;
        uint32_t e[U][8];
        float m[U], x[U], y[U], vx[U], vy[U], Fx[U], Fy[U];
        bool live[U];
        // the blocks' fields, issued before the headers are used
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
            for (int q = 0; q < 8; ++q) e[j][q] = farr<uint32_t>(h, bid[j], p.n_adj + q * p.n_adj_stride)[s];
            m[j] = farr<float>(h, bid[j], p.n_m)[s];
            x[j] = farr<float>(h, bid[j], p.n_x)[s];
            y[j] = farr<float>(h, bid[j], p.n_y)[s];
            vx[j] = farr<float>(h, bid[j], p.n_vx)[s];
            vy[j] = farr<float>(h, bid[j], p.n_vy)[s];
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
            if (px) {
                const uint32_t hd = (bid[j] << 6) | s;
                px[hd] = x[j];
                py[hd] = y[j];
            }
        }
    });
}

template <bool kLoad>
__global__ __launch_bounds__(1024) void k_adj_ckpt(HeapView h, AdjK p)
{
    if (heap_failed(h)) return;
    float *c0 = plane_ptr(p, 4 * p.slot), *c1 = plane_ptr(p, 4 * p.slot + 1);
    float *c2 = plane_ptr(p, 4 * p.slot + 2), *c3 = plane_ptr(p, 4 * p.slot + 3);
    for_each_block(h, p.node_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t hd = (bid << 6) | s;
        float *x = farr<float>(h, bid, p.n_x), *y = farr<float>(h, bid, p.n_y);
        float *vx = farr<float>(h, bid, p.n_vx), *vy = farr<float>(h, bid, p.n_vy);
        if (kLoad) {
            x[s] = c0[hd];
            y[s] = c1[hd];
            vx[s] = c2[hd];
            vy[s] = c3[hd];
        } else {
            c0[hd] = x[s];
            c1[hd] = y[s];
            c2[hd] = vx[s];
            c3[hd] = vy[s];
        }
    });
}

__global__ __launch_bounds__(1024) void k_adj_seed(HeapView h, AdjK p)
{
    for_each_block(h, p.node_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const int32_t id = farr<int32_t>(h, bid, p.n_id)[s];
        if (id < 0 || (uint32_t)id >= p.seed_count) {
            raise_error(h, ERR_BADHANDLE);
            return;
        }
        farr<float>(h, bid, p.n_lx)[s] = p.seed_x[id];
        farr<float>(h, bid, p.n_ly)[s] = p.seed_y[id];
        farr<float>(h, bid, p.n_lvx)[s] = p.seed_vx ? p.seed_vx[id] : 0.f;
        farr<float>(h, bid, p.n_lvy)[s] = p.seed_vy ? p.seed_vy[id] : 0.f;
    });
}

__global__ __launch_bounds__(1024) void k_adj_zero(HeapView h, AdjK p)
{
    for_each_block(h, p.spring_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        farr<float>(h, bid, p.s_gk)[s] = 0.f;
        farr<float>(h, bid, p.s_cx)[s] = 0.f;
        farr<float>(h, bid, p.s_cy)[s] = 0.f;
    });
}

// Node pass: (bit 0) lx, ly += the springs' terms in slot order; (bit 1)
// mu = lv + dt lx, w = mu / m, lv = mu.
__global__ __launch_bounds__(1024) void k_adj_node(HeapView h, AdjK p)
{
    const uint32_t s = lane_id();
    for_each_block_heads<1>(h, p.node_cls, p.wpg, [&](const BlockHeads<1> &hd) {
        const uint32_t bid = hd.bid[0];
        // the node's own fields (the second part's too) and its slots, issued
        // before the header is used and before the gathers of the first part
        float lx = farr<float>(h, bid, p.n_lx)[s], ly = farr<float>(h, bid, p.n_ly)[s];
        const float m = farr<float>(h, bid, p.n_m)[s];
        const float lvx = farr<float>(h, bid, p.n_lvx)[s], lvy = farr<float>(h, bid, p.n_lvy)[s];
        uint32_t e[8];
        if (p.mode & 1u) {
#pragma unroll
            for (int q = 0; q < 8; ++q) e[q] = farr<uint32_t>(h, bid, p.n_adj + q * p.n_adj_stride)[s];
        }
        if (!((hd.bm(0) >> s) & 1)) return;
        if (p.mode & 1u) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (e[q] == kNull) continue;
                const uint32_t sh = e[q] & 0x7FFFFFFFu;
                const float cx = fref<float>(h, sh, p.s_cx), cy = fref<float>(h, sh, p.s_cy);
                if (e[q] >> 31) {
                    lx += cx;
                    ly += cy;
                } else {
                    lx -= cx;
                    ly -= cy;
                }
            }
            farr<float>(h, bid, p.n_lx)[s] = lx;
            farr<float>(h, bid, p.n_ly)[s] = ly;
        }
        if (p.mode & 2u) {
            const float mux = lvx + p.dt * lx;
            const float muy = lvy + p.dt * ly;
            farr<float>(h, bid, p.n_wx)[s] = mux / m;
            farr<float>(h, bid, p.n_wy)[s] = muy / m;
            farr<float>(h, bid, p.n_lvx)[s] = mux;
            farr<float>(h, bid, p.n_lvy)[s] = muy;
        }
    });
}

// Spring pass: c = dt K(x_n) g with g = w_a - w_b, and dL/dk += dt (l - L0) u.g
__global__ __launch_bounds__(1024) void k_adj_spring(HeapView h, AdjK p)
{
    const uint32_t s = lane_id();
    const float *px = plane_ptr(p, 2 * p.slot), *py = plane_ptr(p, 2 * p.slot + 1);
    for_each_block_heads<1>(h, p.spring_cls, p.wpg, [&](const BlockHeads<1> &hd) {
        const uint32_t bid = hd.bid[0];
        // the spring's own fields, issued before the header is used
        const uint32_t a = farr<uint32_t>(h, bid, p.s_a)[s];
        const uint32_t b = farr<uint32_t>(h, bid, p.s_b)[s];
        const float k = farr<float>(h, bid, p.s_k)[s];
        const float L0 = farr<float>(h, bid, p.s_L0)[s];
        if (!((hd.bm(0) >> s) & 1)) return;
        const float dx = px[b] - px[a], dy = py[b] - py[a];
        const float l = sqrtf(dx * dx + dy * dy);
        const float ux = dx / l, uy = dy / l;
        const float gx = fref<float>(h, a, p.n_wx) - fref<float>(h, b, p.n_wx);
        const float gy = fref<float>(h, a, p.n_wy) - fref<float>(h, b, p.n_wy);
        const float ug = ux * gx + uy * gy;
        const float r = L0 / l;
        const float kgx = k * ((1.f - r) * gx + r * ux * ug);
        const float kgy = k * ((1.f - r) * gy + r * uy * ug);
        farr<float>(h, bid, p.s_cx)[s] = p.dt * kgx;
        farr<float>(h, bid, p.s_cy)[s] = p.dt * kgy;
        farr<float>(h, bid, p.s_gk)[s] += p.dt * (l - L0) * ug;
    });
}

smmo_status bind_adj(smmo_heap *h, const AdjKey &key, AdjK &k)
{
    const uint32_t nc = h->schema->nclasses;
    if (key.node_class >= nc || key.spring_class >= nc || key.node_class == key.spring_class)
        return fail(SMMO_EINVAL, "adjoint: bad class ids");
    k.node_cls = key.node_class;
    k.spring_cls = key.spring_class;
    const uint32_t N = key.node_class, S = key.spring_class;
    BIND(N, "x", SMMO_F32, 1, &k.n_x, nullptr);
    BIND(N, "y", SMMO_F32, 1, &k.n_y, nullptr);
    BIND(N, "vx", SMMO_F32, 1, &k.n_vx, nullptr);
    BIND(N, "vy", SMMO_F32, 1, &k.n_vy, nullptr);
    BIND(N, "m", SMMO_F32, 1, &k.n_m, nullptr);
    BIND(N, "adj", SMMO_HANDLE, 8, &k.n_adj, &k.n_adj_stride);
    BIND(N, "id", SMMO_I32, 1, &k.n_id, nullptr);
    BIND(N, "lx", SMMO_F32, 1, &k.n_lx, nullptr);
    BIND(N, "ly", SMMO_F32, 1, &k.n_ly, nullptr);
    BIND(N, "lvx", SMMO_F32, 1, &k.n_lvx, nullptr);
    BIND(N, "lvy", SMMO_F32, 1, &k.n_lvy, nullptr);
    BIND(N, "wx", SMMO_F32, 1, &k.n_wx, nullptr);
    BIND(N, "wy", SMMO_F32, 1, &k.n_wy, nullptr);
    BIND(S, "a", SMMO_HANDLE, 1, &k.s_a, nullptr);
    BIND(S, "b", SMMO_HANDLE, 1, &k.s_b, nullptr);
    BIND(S, "k", SMMO_F32, 1, &k.s_k, nullptr);
    BIND(S, "L0", SMMO_F32, 1, &k.s_L0, nullptr);
    BIND(S, "cx", SMMO_F32, 1, &k.s_cx, nullptr);
    BIND(S, "cy", SMMO_F32, 1, &k.s_cy, nullptr);
    BIND(S, "gk", SMMO_F32, 1, &k.s_gk, nullptr);
    BIND(S, "fx", SMMO_F32, 1, &k.s_fx, nullptr);
    BIND(S, "fy", SMMO_F32, 1, &k.s_fy, nullptr);
    return SMMO_OK;
}

enum Which { W_RECORD, W_SAVE, W_LOAD, W_SEED, W_ZERO, W_NODE, W_SPRING, W_STEP };

// blocks per wavefront iteration of the forward node pass unless set otherwise
constexpr uint32_t kStepGroup = 1;

template <int Which>
smmo_status launch_adj(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_adjoint_args a;
    memcpy(&a, args, sizeof a);
    const AdjKey key{a.node_class, a.spring_class};
    AdjK k;
    smmo_status s = cached_bind(h, (const void *)&launch_adj<W_NODE>, 0u, key, k,
                                [&] { return bind_adj(h, key, k); });
    if (s) return s;
    const bool on_spring = Which == W_ZERO || Which == W_SPRING;
    if (cls != (on_spring ? a.spring_class : a.node_class))
        return fail(SMMO_EINVAL, "adjoint: method runs on a different class");
    if (!(a.dt == a.dt)) return fail(SMMO_EINVAL, "adjoint: dt is NaN");
    k.dt = a.dt;
    k.mode = a.mode;
    k.tape = a.tape;
    k.plane = a.plane;
    k.slot = a.slot;
    k.seed_count = a.seed_count;
    k.seed_x = a.seed_x;
    k.seed_y = a.seed_y;
    k.seed_vx = a.seed_vx;
    k.seed_vy = a.seed_vy;
    const uint32_t planes = (Which == W_SAVE || Which == W_LOAD) ? 4u : 2u;
    if (Which == W_RECORD || Which == W_SAVE || Which == W_LOAD || Which == W_SPRING ||
        (Which == W_STEP && a.tape)) {
        if (!a.tape) return fail(SMMO_EINVAL, "adjoint: tape is NULL");
        if (a.plane < 64ull * h->v.M) return fail(SMMO_EINVAL, "adjoint: tape plane shorter than 64 * heap blocks");
        if (((uint64_t)a.slot + 1) * planes * a.plane > a.tape_floats)
            return fail(SMMO_EINVAL, "adjoint: tape slot beyond the tape's capacity");
    }
    if (Which == W_SEED && (!a.seed_x || !a.seed_y)) return fail(SMMO_EINVAL, "adjoint: seed arrays are NULL");
    if (Which == W_NODE && (a.mode & ~3u)) return fail(SMMO_EINVAL, "adjoint: bad mode");
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    if (Which == W_STEP) {
        const LaunchShape ls = method_shape(h, cls, kStepGroup);
        k.wpg = ls.block.x / 64;
        if (ls.group == 4) hipLaunchKernelGGL(k_adj_step_node<4>, ls.grid, ls.block, 0, st, h->v, k);
        else if (ls.group == 2) hipLaunchKernelGGL(k_adj_step_node<2>, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_adj_step_node<1>, ls.grid, ls.block, 0, st, h->v, k);
        return launched("adjoint kernel");
    }
    const LaunchShape ls = method_shape(h, cls);
    k.wpg = ls.block.x / 64;
    const dim3 grid = ls.grid, blk = ls.block;
    switch (Which) {
    case W_RECORD: hipLaunchKernelGGL(k_adj_record, grid, blk, 0, st, h->v, k); break;
    case W_SAVE: hipLaunchKernelGGL(k_adj_ckpt<false>, grid, blk, 0, st, h->v, k); break;
    case W_LOAD: hipLaunchKernelGGL(k_adj_ckpt<true>, grid, blk, 0, st, h->v, k); break;
    case W_SEED: hipLaunchKernelGGL(k_adj_seed, grid, blk, 0, st, h->v, k); break;
    case W_ZERO: hipLaunchKernelGGL(k_adj_zero, grid, blk, 0, st, h->v, k); break;
    case W_NODE: hipLaunchKernelGGL(k_adj_node, grid, blk, 0, st, h->v, k); break;
    case W_SPRING: hipLaunchKernelGGL(k_adj_spring, grid, blk, 0, st, h->v, k); break;
    }
    return launched("adjoint kernel");
}

} // namespace

namespace smmo {
smmo_status launch_adj_record(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_RECORD>(h, c, a, s); }
smmo_status launch_adj_save(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_SAVE>(h, c, a, s); }
smmo_status launch_adj_load(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_LOAD>(h, c, a, s); }
smmo_status launch_adj_seed(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_SEED>(h, c, a, s); }
smmo_status launch_adj_zero(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_ZERO>(h, c, a, s); }
smmo_status launch_adj_node(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_NODE>(h, c, a, s); }
smmo_status launch_adj_spring(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_SPRING>(h, c, a, s); }
smmo_status launch_adj_step_node(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_adj<W_STEP>(h, c, a, s); }
} // namespace smmo
