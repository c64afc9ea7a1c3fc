// wa-tor (Ch.7 "wa-tor"): fish and sharks on a torus of cells, eight do-alls
// per iteration (field contracts in include/smmo_methods.h).
//
// Agents move without atomics, as in the thesis: an agent marks a request
// byte in the target cell (one byte per direction, so concurrent requests
// touch different bytes), every cell grants one request, and the granted
// agents move.  Fish and sharks are created (spawn) and deleted (eaten,
// starved) inside the update methods through the device allocator.  Random
// choices use a counter-based generator keyed by (iteration, phase, cell), so
// they do not depend on thread order or object placement.
#include <hip/hip_runtime.h>

#include <cstring>

#include "method_common.hpp"

using namespace smmo;

namespace {

constexpr uint32_t kShark = 0x80000000u;   // tag of a Shark handle in Cell::agent

struct WatorK {
    uint32_t cell_cls, fish_cls, shark_cls;
    uint32_t t;
    uint64_t seed;
    int32_t fish_spawn, shark_spawn, energy0, boost;
    uint32_t kind;
    int32_t W, H;
    const uint32_t *cells;
    // Cell fields
    uint32_t c_agent, c_nb, c_nb_stride, c_req, c_req_stride, c_id;
    // Fish fields
    uint32_t f_pos, f_new, f_timer;
    // Shark fields
    uint32_t s_pos, s_new, s_timer, s_energy;
};

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014) in counter mode: the
// output function applied to seed + gamma * (counter + 1)
__device__ __forceinline__ uint64_t wt_random(uint64_t seed, uint32_t stream, uint32_t idx)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((((uint64_t)stream) << 32) + idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t self_handle(uint32_t bid) { return (bid << 6) | lane_id(); }

// a handle read from a field that other methods write: names a block of the
// heap (else the device error is set and the caller skips the access)
__device__ __forceinline__ bool wt_valid(const HeapView &h, uint32_t handle)
{
    if ((handle >> 6) < h.M) return true;
    raise_error(h, ERR_INTERNAL);
    return false;
}

// Cell::prepare
__global__ __launch_bounds__(1024) void k_wt_cell_prepare(HeapView h, WatorK p)
{
    for_each_block(h, p.cell_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
#pragma unroll
        for (int q = 0; q < 5; ++q) farr<uint8_t>(h, bid, p.c_req + q * p.c_req_stride)[s] = 0;
    });
}

// An agent on cell c asks to enter one neighbour: among those whose agent
// passes `first` (tried first) or, if none, `second`, one at random; with no
// candidate it asks to stay.  0 = empty, 1 = fish, 2 = never.
__device__ __forceinline__ bool wt_kind_is(uint32_t agent, uint32_t want)
{
    if (want == 0) return agent == kNull;
    if (want == 1) return agent != kNull && !(agent & kShark);
    return false;
}

__device__ __forceinline__ void wt_request(const HeapView &h, const WatorK &p, uint32_t c, uint32_t first,
                                           uint32_t second, uint32_t stream)
{
    uint32_t nb[4], ag[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nb[q] = fref<uint32_t>(h, c, p.c_nb + q * p.c_nb_stride);
#pragma unroll
    for (int q = 0; q < 4; ++q) ag[q] = wt_valid(h, nb[q]) ? fref<uint32_t>(h, nb[q], p.c_agent) : kShark;
    // candidate directions as a bit mask, in direction order
    uint32_t mask = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) mask |= wt_kind_is(ag[q], first) ? 1u << q : 0u;
    if (mask == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) mask |= wt_kind_is(ag[q], second) ? 1u << q : 0u;
    }
    if (mask == 0) {
        fref<uint8_t>(h, c, p.c_req + 4 * p.c_req_stride) = 1;
        return;
    }
    const uint32_t cid = (uint32_t)fref<int32_t>(h, c, p.c_id);
    const uint32_t k = (uint32_t)(wt_random(p.seed, stream, cid) % (uint64_t)__popc(mask));
    const uint32_t sel = nth_set_bit(mask, k);
    uint32_t target = nb[0];
#pragma unroll
    for (int q = 1; q < 4; ++q)
        if ((uint32_t)q == sel) target = nb[q];
    fref<uint8_t>(h, target, p.c_req + ((sel + 2) & 3) * p.c_req_stride) = 1;
}

// Fish::prepare
__global__ __launch_bounds__(1024) void k_wt_fish_prepare(HeapView h, WatorK p)
{
    for_each_object_packed(h, p.fish_cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        if (!live) return;
        int32_t &timer = farr<int32_t>(h, bid, p.f_timer)[s];
        timer += 1;
        const uint32_t pos = farr<uint32_t>(h, bid, p.f_pos)[s];
        farr<uint32_t>(h, bid, p.f_new)[s] = pos;
        if (wt_valid(h, pos)) wt_request(h, p, pos, 0, 2, 4 * p.t + 0);
    });
}

// Shark::prepare
__global__ __launch_bounds__(1024) void k_wt_shark_prepare(HeapView h, WatorK p)
{
    for_each_object_packed(h, p.shark_cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        if (!live) return;
        farr<int32_t>(h, bid, p.s_timer)[s] += 1;
        farr<int32_t>(h, bid, p.s_energy)[s] -= 1;
        const uint32_t pos = farr<uint32_t>(h, bid, p.s_pos)[s];
        farr<uint32_t>(h, bid, p.s_new)[s] = pos;
        if (wt_valid(h, pos)) wt_request(h, p, pos, 1, 0, 4 * p.t + 2);
    });
}

// Cell::decide for the agents of class p.kind (1 fish, 2 shark)
__global__ __launch_bounds__(1024) void k_wt_cell_decide(HeapView h, WatorK p)
{
    if (heap_failed(h)) return;
    const uint32_t o_new = p.kind == 1 ? p.f_new : p.s_new;
    const uint32_t stream = 4 * p.t + (p.kind == 1 ? 1u : 3u);
    for_each_block(h, p.cell_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        uint8_t rq[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) rq[q] = farr<uint8_t>(h, bid, p.c_req + q * p.c_req_stride)[s];
        const uint32_t me = self_handle(bid);
        if (rq[4]) {
            const uint32_t a = farr<uint32_t>(h, bid, p.c_agent)[s] & ~kShark;
            if (wt_valid(h, a)) fref<uint32_t>(h, a, o_new) = me;
            return;
        }
        uint32_t mask = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) mask |= rq[q] ? 1u << q : 0u;
        if (mask == 0) return;
        const uint32_t cid = (uint32_t)farr<int32_t>(h, bid, p.c_id)[s];
        const uint32_t k = (uint32_t)(wt_random(p.seed, stream, cid) % (uint64_t)__popc(mask));
        const uint32_t sel = nth_set_bit(mask, k);
        const uint32_t o = farr<uint32_t>(h, bid, p.c_nb + sel * p.c_nb_stride)[s];
        if (!wt_valid(h, o)) return;
        const uint32_t a = fref<uint32_t>(h, o, p.c_agent) & ~kShark;
        if (wt_valid(h, a)) fref<uint32_t>(h, a, o_new) = me;
    });
}

// Fish::update (the iteration snapshot keeps new fish out of this launch)
__global__ __launch_bounds__(1024) void k_wt_fish_update(HeapView h, WatorK p)
{
    for_each_object_packed(h, p.fish_cls, true, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        uint32_t pos = 0, np = 0;
        int32_t timer = 0;
        if (live) {
            pos = farr<uint32_t>(h, bid, p.f_pos)[s];
            np = farr<uint32_t>(h, bid, p.f_new)[s];
            timer = farr<int32_t>(h, bid, p.f_timer)[s];
        }
        const bool moved = live && np != pos && wt_valid(h, np) && wt_valid(h, pos);
        if (moved) {
            fref<uint32_t>(h, np, p.c_agent) = (bid << 6) | s;
            farr<uint32_t>(h, bid, p.f_pos)[s] = np;
        }
        const bool spawn = moved && timer > p.fish_spawn;
        const uint32_t child = wave_allocate(h, p.fish_cls, spawn);
        if (spawn && child != kNull) {
            fref<uint32_t>(h, child, p.f_pos) = pos;
            fref<uint32_t>(h, child, p.f_new) = pos;
            fref<int32_t>(h, child, p.f_timer) = 0;
            farr<int32_t>(h, bid, p.f_timer)[s] = 0;
        }
        if (moved) fref<uint32_t>(h, pos, p.c_agent) = spawn ? child : kNull;
    });
}

// Shark::update (snapshot as above); a starving shark deletes itself last
__global__ __launch_bounds__(1024) void k_wt_shark_update(HeapView h, WatorK p)
{
    for_each_object_packed(h, p.shark_cls, true, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        uint32_t pos = 0, np = 0;
        int32_t timer = 0, energy = 0;
        if (live) {
            pos = farr<uint32_t>(h, bid, p.s_pos)[s];
            np = farr<uint32_t>(h, bid, p.s_new)[s];
            timer = farr<int32_t>(h, bid, p.s_timer)[s];
            energy = farr<int32_t>(h, bid, p.s_energy)[s];
        }
        const bool die = live && energy <= 0;
        if (die && wt_valid(h, pos)) fref<uint32_t>(h, pos, p.c_agent) = kNull;
        const bool moved = live && !die && np != pos && wt_valid(h, np) && wt_valid(h, pos);
        uint32_t prey = kNull;
        if (moved) {
            prey = fref<uint32_t>(h, np, p.c_agent);
            if (prey != kNull && ((prey & kShark) || !wt_valid(h, prey))) {
                raise_error(h, ERR_INTERNAL);   // a granted target never holds a shark
                prey = kNull;
            }
            if (prey != kNull) farr<int32_t>(h, bid, p.s_energy)[s] = energy + p.boost;
            fref<uint32_t>(h, np, p.c_agent) = (bid << 6) | s | kShark;
            farr<uint32_t>(h, bid, p.s_pos)[s] = np;
        }
        wave_deallocate(h, p.fish_cls, prey, prey != kNull);
        const bool spawn = moved && timer > p.shark_spawn;
        const uint32_t child = wave_allocate(h, p.shark_cls, spawn);
        if (spawn && child != kNull) {
            fref<uint32_t>(h, child, p.s_pos) = pos;
            fref<uint32_t>(h, child, p.s_new) = pos;
            fref<int32_t>(h, child, p.s_timer) = 0;
            fref<int32_t>(h, child, p.s_energy) = p.energy0;
            farr<int32_t>(h, bid, p.s_timer)[s] = 0;
        }
        if (moved) fref<uint32_t>(h, pos, p.c_agent) = spawn && child != kNull ? child | kShark : kNull;
        wave_release_packed(h, p.shark_cls, bid, s, die, pair);
    });
}

// Cell::link - neighbours from the cell index on the torus
__global__ __launch_bounds__(1024) void k_wt_cell_link(HeapView h, WatorK p)
{
    for_each_block(h, p.cell_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const int32_t id = farr<int32_t>(h, bid, p.c_id)[s];
        if (id < 0 || id >= p.W * p.H) {
            raise_error(h, ERR_BADHANDLE);
            return;
        }
        const int32_t x = id % p.W, y = id / p.W;
        const int32_t nid[4] = {((y - 1 + p.H) % p.H) * p.W + x, y * p.W + (x + 1) % p.W,
                                ((y + 1) % p.H) * p.W + x, y * p.W + (x - 1 + p.W) % p.W};
#pragma unroll
        for (int q = 0; q < 4; ++q) farr<uint32_t>(h, bid, p.c_nb + q * p.c_nb_stride)[s] = p.cells[nid[q]];
    });
}

// Agent::link - its cell's agent field names it
__global__ __launch_bounds__(1024) void k_wt_link(HeapView h, WatorK p)
{
    if (heap_failed(h)) return;
    const uint32_t cls = p.kind == 1 ? p.fish_cls : p.shark_cls;
    const uint32_t o_pos = p.kind == 1 ? p.f_pos : p.s_pos;
    const uint32_t tag = p.kind == 1 ? 0u : kShark;
    for_each_block(h, cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const uint32_t pos = farr<uint32_t>(h, bid, o_pos)[s];
        if (wt_valid(h, pos)) fref<uint32_t>(h, pos, p.c_agent) = self_handle(bid) | tag;
    });
}

smmo_status bind_wator(smmo_heap *h, const smmo_wator_args &a, WatorK &k)
{
    const uint32_t nc = h->schema->nclasses;
    if (a.cell_class >= nc || a.fish_class >= nc || a.shark_class >= nc || a.cell_class == a.fish_class ||
        a.cell_class == a.shark_class || a.fish_class == a.shark_class)
        return fail(SMMO_EINVAL, "wator: bad class ids");
    memset(&k, 0, sizeof k);
    k.cell_cls = a.cell_class;
    k.fish_cls = a.fish_class;
    k.shark_cls = a.shark_class;
    BIND(a.cell_class, "agent", SMMO_HANDLE, 1, &k.c_agent, nullptr);
    BIND(a.cell_class, "nb", SMMO_HANDLE, 4, &k.c_nb, &k.c_nb_stride);
    BIND(a.cell_class, "req", SMMO_U8, 5, &k.c_req, &k.c_req_stride);
    BIND(a.cell_class, "cell_id", SMMO_I32, 1, &k.c_id, nullptr);
    BIND(a.fish_class, "pos", SMMO_HANDLE, 1, &k.f_pos, nullptr);
    BIND(a.fish_class, "new_pos", SMMO_HANDLE, 1, &k.f_new, nullptr);
    BIND(a.fish_class, "timer", SMMO_I32, 1, &k.f_timer, nullptr);
    BIND(a.shark_class, "pos", SMMO_HANDLE, 1, &k.s_pos, nullptr);
    BIND(a.shark_class, "new_pos", SMMO_HANDLE, 1, &k.s_new, nullptr);
    BIND(a.shark_class, "timer", SMMO_I32, 1, &k.s_timer, nullptr);
    BIND(a.shark_class, "energy", SMMO_I32, 1, &k.s_energy, nullptr);
    return SMMO_OK;
}

// Which: 0 cell_prepare, 1 fish_prepare, 2 shark_prepare, 3 cell_decide,
// 4 fish_update, 5 shark_update, 6 cell_link, 7 link
template <int Which>
smmo_status launch_wator(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_wator_args a;
    memcpy(&a, args, sizeof a);
    // the per-call fields do not take part in the binding
    smmo_wator_args key = a;
    key.iteration = 0;
    key.seed = 0;
    key.fish_spawn = key.shark_spawn = key.energy0 = key.boost = 0;
    key.kind = 0;
    key.width = key.height = 0;
    key.cells = nullptr;
    WatorK k;
    smmo_status s = cached_bind(h, (const void *)&launch_wator<0>, cls, key, k,
                                [&] { return bind_wator(h, a, k); });
    if (s) return s;
    k.t = a.iteration;
    k.seed = a.seed;
    k.fish_spawn = a.fish_spawn;
    k.shark_spawn = a.shark_spawn;
    k.energy0 = a.energy0;
    k.boost = a.boost;
    k.kind = a.kind;
    k.W = a.width;
    k.H = a.height;
    k.cells = a.cells;
    uint32_t want = a.cell_class;
    if (Which == 1 || Which == 4) want = a.fish_class;
    if (Which == 2 || Which == 5) want = a.shark_class;
    if (Which == 7) {
        if (a.kind != 1 && a.kind != 2) return fail(SMMO_EINVAL, "wator.link: kind must be 1 or 2");
        want = a.kind == 1 ? a.fish_class : a.shark_class;
    }
    if (cls != want) return fail(SMMO_EINVAL, "wator: method runs on a different class");
    if (Which == 3 && a.kind != 1 && a.kind != 2) return fail(SMMO_EINVAL, "wator.cell_decide: kind must be 1 or 2");
    if (Which == 6 && (!a.cells || a.width <= 0 || a.height <= 0 ||
                       (int64_t)a.width * a.height > 0x7FFFFFFF))
        return fail(SMMO_EINVAL, "wator.cell_link: bad grid");
    const bool snapshot = Which == 4 || Which == 5;
    // the agent classes (fragmented by births and deaths) run packed do-alls,
    // packed as the heap's sparse_packing setting asks
    const bool packed = Which == 1 || Which == 2 || Which == 4 || Which == 5;
    const LaunchShape ls = method_shape(h, cls);
    if ((s = ensure_enumerated(h, cls, snapshot, st, packed && packing_wanted(h, cls, ls)))) return s;
    switch (Which) {
    case 0: hipLaunchKernelGGL(k_wt_cell_prepare, ls.grid, ls.block, 0, st, h->v, k); break;
    case 1: hipLaunchKernelGGL(k_wt_fish_prepare, ls.grid, ls.block, 0, st, h->v, k); break;
    case 2: hipLaunchKernelGGL(k_wt_shark_prepare, ls.grid, ls.block, 0, st, h->v, k); break;
    case 3: hipLaunchKernelGGL(k_wt_cell_decide, ls.grid, ls.block, 0, st, h->v, k); break;
    case 4: hipLaunchKernelGGL(k_wt_fish_update, ls.grid, ls.block, 0, st, h->v, k); break;
    case 5: hipLaunchKernelGGL(k_wt_shark_update, ls.grid, ls.block, 0, st, h->v, k); break;
    case 6: hipLaunchKernelGGL(k_wt_cell_link, ls.grid, ls.block, 0, st, h->v, k); break;
    default: hipLaunchKernelGGL(k_wt_link, ls.grid, ls.block, 0, st, h->v, k); break;
    }
    if ((s = launched("wator kernel"))) return s;
    // a fish update can create up to one fish per fish; a shark update one
    // shark per shark
    if (Which == 4) note_allocation(h, a.fish_class, 64ull * h->ub_blocks[a.fish_class]);
    if (Which == 5) note_allocation(h, a.shark_class, 64ull * h->ub_blocks[a.shark_class]);
    return SMMO_OK;
}

} // namespace

namespace smmo {
smmo_status launch_wator_cell_prepare(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<0>(h, c, a, s); }
smmo_status launch_wator_fish_prepare(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<1>(h, c, a, s); }
smmo_status launch_wator_shark_prepare(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<2>(h, c, a, s); }
smmo_status launch_wator_cell_decide(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<3>(h, c, a, s); }
smmo_status launch_wator_fish_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<4>(h, c, a, s); }
smmo_status launch_wator_shark_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<5>(h, c, a, s); }
smmo_status launch_wator_cell_link(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<6>(h, c, a, s); }
smmo_status launch_wator_link(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_wator<7>(h, c, a, s); }
} // namespace smmo
