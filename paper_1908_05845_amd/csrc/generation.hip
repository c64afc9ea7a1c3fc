// generation (Ch.7 "generation"): Game of Life with dying cells on a torus,
// in the Cell + Alive form of the Game of Life here (field contracts in
// include/smmo_methods.h).  An Alive object lives from its cell's birth until
// the end of the cell's dying period; births are device allocations in
// Cell::birth, deletions self-deletions in Alive::update.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

using namespace smmo;

namespace {

struct GenK {
    uint32_t cell_cls, alive_cls;
    const uint32_t *cells;
    int32_t W, H;
    uint32_t survive, birth;
    int32_t dying;
    uint32_t c_state, c_count, c_id;   // Cell fields
    uint32_t a_id, a_left, a_new;      // Alive fields
};

// a Cell handle from the caller's grid array names a block of the heap
__device__ __forceinline__ bool gen_valid(const HeapView &h, uint32_t handle)
{
    if ((handle >> 6) < h.M) return true;
    raise_error(h, ERR_BADHANDLE);
    return false;
}

// Cell::count - live neighbours on the torus (dying cells do not count).
// One integer division per cell, neighbour wrap-around by compare and select,
// two blocks per wavefront iteration (as the Game of Life's count).
template <int U>
__global__ __launch_bounds__(1024) void k_gen_count(HeapView h, GenK p)
{
    const uint32_t s = lane_id();
    bool bad = false;                  // a cell id outside the grid or a handle outside the heap
    for_each_block_group<U>(h, p.cell_cls, [&](const uint32_t *bid, const uint64_t *bm, const bool *own) {
        bool live[U];
        int32_t id[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            live[j] = (bm[j] >> s) & 1;
            id[j] = live[j] ? farr<int32_t>(h, bid[j], p.c_id)[s] : 0;
            if (live[j] && (uint32_t)id[j] >= (uint32_t)(p.W * p.H)) {
                bad = true;                        // a cell id outside the grid
                live[j] = false;
            }
        }
        uint32_t hc[U][8];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t y = id[j] / p.W, x = id[j] - y * p.W;
            const int32_t xs[3] = {x == 0 ? p.W - 1 : x - 1, x, x == p.W - 1 ? 0 : x + 1};
            const int32_t rows[3] = {(y == 0 ? p.H - 1 : y - 1) * p.W, y * p.W,
                                     (y == p.H - 1 ? 0 : y + 1) * p.W};
            int k = 0;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    if (dx == 1 && dy == 1) continue;
                    uint32_t c = live[j] ? p.cells[rows[dy] + xs[dx]] : 0u;
                    if ((c >> 6) >= h.M) {          // not a handle of this heap: read block 0 instead
                        bad = true;
                        c = 0;
                    }
                    hc[j][k++] = c;
                }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!own[j] || !live[j]) continue;
            int32_t n = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) n += fref<uint8_t>(h, hc[j][k], p.c_state) == 1;
            farr<int32_t>(h, bid[j], p.c_count)[s] = n;
        }
    });
    // reported once, after the walk
    if (__ballot(bad) && s == (uint32_t)(__ffsll((unsigned long long)__ballot(bad)) - 1))
        raise_error(h, ERR_BADHANDLE);
}

// Cell::birth - an empty cell with a count in the birth set comes alive
__global__ __launch_bounds__(1024) void k_gen_birth(HeapView h, GenK p)
{
    for_each_block(h, p.cell_cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        // a view of the Alive class's active blocks, loaded beside the fields
        const ActiveView view = active_view(h, p.alive_cls);
        bool born = false;
        int32_t id = 0;
        if ((bm >> s) & 1) {
            uint8_t &st = farr<uint8_t>(h, bid, p.c_state)[s];
            if (st == 0 && ((p.birth >> farr<int32_t>(h, bid, p.c_count)[s]) & 1)) {
                st = 1;
                born = true;
                id = farr<int32_t>(h, bid, p.c_id)[s];
            }
        }
        const uint32_t a = wave_allocate(h, p.alive_cls, born, &view);
        if (born && a != kNull) {
            fref<int32_t>(h, a, p.a_id) = id;
            fref<int32_t>(h, a, p.a_left) = 0;
            fref<uint8_t>(h, a, p.a_new) = 1;
        }
    });
}

// Alive::update - survive or start dying; count a dying period down and
// delete this at its end
__global__ __launch_bounds__(1024) void k_gen_alive_update(HeapView h, GenK p)
{
    for_each_object_packed(h, p.alive_cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        bool gone = false;
        const int32_t cid = live ? farr<int32_t>(h, bid, p.a_id)[s] : 0;
        if (live && ((uint32_t)cid >= (uint32_t)(p.W * p.H) || !gen_valid(h, p.cells[cid]))) {
            raise_error(h, ERR_BADHANDLE);
            live = false;
        }
        if (live) {
            uint8_t &fresh = farr<uint8_t>(h, bid, p.a_new)[s];
            int32_t &left = farr<int32_t>(h, bid, p.a_left)[s];
            const uint32_t hc = p.cells[cid];
            if (fresh) {
                fresh = 0;
            } else if (left == 0) {
                if (!((p.survive >> fref<int32_t>(h, hc, p.c_count)) & 1)) {
                    left = p.dying;
                    fref<uint8_t>(h, hc, p.c_state) = 2;
                }
            } else if (--left == 0) {
                fref<uint8_t>(h, hc, p.c_state) = 0;
                gone = true;
            }
        }
        wave_release_packed(h, p.alive_cls, bid, s, gone, pair);
    });
}

smmo_status bind_generation(smmo_heap *h, const smmo_generation_args &a, GenK &k)
{
    const uint32_t nc = h->schema->nclasses;
    if (a.cell_class >= nc || a.alive_class >= nc || a.cell_class == a.alive_class)
        return fail(SMMO_EINVAL, "generation: bad class ids");
    if (!a.cells || a.width <= 0 || a.height <= 0 || (int64_t)a.width * a.height > 0x7FFFFFFF)
        return fail(SMMO_EINVAL, "generation: bad grid");
    if (a.dying < 1 || (a.survive >> 9) || (a.birth >> 9))
        return fail(SMMO_EINVAL, "generation: rule masks cover the counts 0..8 and dying must be >= 1");
    k.cell_cls = a.cell_class;
    k.alive_cls = a.alive_class;
    k.cells = a.cells;
    k.W = a.width;
    k.H = a.height;
    k.survive = a.survive;
    k.birth = a.birth;
    k.dying = a.dying;
    BIND(a.cell_class, "state", SMMO_U8, 1, &k.c_state, nullptr);
    BIND(a.cell_class, "count", SMMO_I32, 1, &k.c_count, nullptr);
    BIND(a.cell_class, "cell_id", SMMO_I32, 1, &k.c_id, nullptr);
    BIND(a.alive_class, "cell_id", SMMO_I32, 1, &k.a_id, nullptr);
    BIND(a.alive_class, "left", SMMO_I32, 1, &k.a_left, nullptr);
    BIND(a.alive_class, "is_new", SMMO_U8, 1, &k.a_new, nullptr);
    return SMMO_OK;
}

// blocks per wavefront iteration of Cell::count unless set otherwise
constexpr uint32_t kGenCountGroup = 2;

// Which: 0 cell_count, 1 cell_birth, 2 alive_update
template <int Which>
smmo_status launch_generation(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_generation_args a;
    memcpy(&a, args, sizeof a);
    GenK k;
    smmo_status s = cached_bind(h, (const void *)&launch_generation<0>, cls, a, k,
                                [&] { return bind_generation(h, a, k); });
    if (s) return s;
    const uint32_t want = Which == 2 ? a.alive_class : a.cell_class;
    if (cls != want) return fail(SMMO_EINVAL, "generation: method runs on a different class");
    const LaunchShape ls = method_shape(h, cls, Which == 0 ? kGenCountGroup : 0);
    if ((s = ensure_enumerated(h, cls, false, st, Which == 2 && packing_wanted(h, cls, ls)))) return s;
    if (Which == 0) {
        if (ls.group == 4) hipLaunchKernelGGL(k_gen_count<4>, ls.grid, ls.block, 0, st, h->v, k);
        else if (ls.group == 2) hipLaunchKernelGGL(k_gen_count<2>, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_gen_count<1>, ls.grid, ls.block, 0, st, h->v, k);
    }
    if (Which == 1) hipLaunchKernelGGL(k_gen_birth, ls.grid, ls.block, 0, st, h->v, k);
    if (Which == 2) hipLaunchKernelGGL(k_gen_alive_update, ls.grid, ls.block, 0, st, h->v, k);
    if ((s = launched("generation kernel"))) return s;
    if (Which == 1) note_allocation(h, a.alive_class, 64ull * h->v.M);
    return SMMO_OK;
}

} // namespace

namespace smmo {
smmo_status launch_generation_cell_count(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_generation<0>(h, c, a, s); }
smmo_status launch_generation_cell_birth(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_generation<1>(h, c, a, s); }
smmo_status launch_generation_alive_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_generation<2>(h, c, a, s); }
} // namespace smmo
