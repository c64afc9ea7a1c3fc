// Methods that smmo_parallel_do() can run: Game of Life, n-body, the test
// methods and the allocator microbenchmark (argument structs and field
// contracts in include/smmo_methods.h; the spring-mass methods are in
// spring.hip, wa-tor in wator.hip, the adjoint in adjoint.hip).
//
// Every method kernel walks the class's block list R (built by the
// enumeration pre-pass) with one wavefront per block and one lane per slot,
// the thread assignment of DynaSOAr's parallel_do with N_T = 64 (Ch.5
// sec.5.2.7): lane s handles slot s, so each field access of a wavefront is
// one contiguous 64-entry run.  The launch is a fixed grid that strides over
// R, whose length is read on the device, so step loops need no host
// read-back.  Work-groups are renumbered so that each of the eight XCDs
// (each with its own L2) walks a contiguous stretch of R.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "../../include/smmo_methods.h"
#include "method_common.hpp"

using namespace smmo;

namespace {

// ======================================================= Game of Life =====
struct GolK {
    uint32_t cell_cls, alive_cls;
    const uint32_t *cells;
    int32_t W, H;
    uint32_t c_state, c_count, c_id;   // Cell field offsets
    uint32_t a_id;                     // Alive field offset
    uint32_t wpg;                      // wavefronts per work-group of this launch
    uint32_t snap;                     // Cell::count: also take the Alive snapshot of every block
    uint32_t death_groups;             // fused generation: work-groups that run Alive::death
};

// a Cell handle from the caller's grid array names a block of the heap
__device__ __forceinline__ bool gol_valid(const HeapView &h, uint32_t handle)
{
    if ((handle >> 6) < h.M) return true;
    raise_error(h, ERR_BADHANDLE);
    return false;
}

// Cell::count - live cells among the 8 neighbours on the torus.  One
// integer division per cell (gfx950 has no integer divide instruction); the
// wrap-around of the neighbour coordinates is a compare and select.  U
// blocks at once: a wavefront issues the neighbour-handle loads and then the
// state loads of all U blocks before it waits, since each block's chain of
// dependent loads (cell id, handles, states) is what bounds the walk.
template <int U>
__global__ __launch_bounds__(1024) void k_gol_count(HeapView h, GolK p)
{
    const uint32_t s = lane_id();
    if (p.snap) {
        // the Alive snapshot of the fused death and birth launch that
        // follows: every block's iteration bitmap, zero for blocks of other
        // classes (a block that becomes an Alive block in that launch then
        // lists nothing).  Nothing allocates or releases during this pass.
        const uint32_t n = gridDim.x * blockDim.x;
        for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < h.M; b += n)
            h.iter_bm[b] = h.type[b] == p.alive_cls ? h.alloc_bm[b] : 0ull;
    }
    bool bad = false;                  // a cell id outside the grid or a handle outside the heap
    for_each_block_heads<U>(h, p.cell_cls, p.wpg, [&](const BlockHeads<U> &hd) {
        const uint32_t *bid = hd.bid;
        bool live[U];
        int32_t id[U];
        // the cell ids, issued before the headers are used
#pragma unroll
        for (int j = 0; j < U; ++j) id[j] = farr<int32_t>(h, bid[j], p.c_id)[s];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            live[j] = (hd.bm(j) >> s) & 1;
            if (!live[j]) id[j] = 0;
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
            if (!hd.own(j)) continue;
            int32_t n = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (live[j]) n += fref<uint8_t>(h, hc[j][k], p.c_state);
            if (live[j]) farr<int32_t>(h, bid[j], p.c_count)[s] = n;
        }
    });
    // reported once, after the walk
    if (__ballot(bad) && s == (uint32_t)(__ffsll((unsigned long long)__ballot(bad)) - 1))
        raise_error(h, ERR_BADHANDLE);
}

// Alive::death - if the cell's count is not 2 or 3: cell dies, delete this
// (a packed do-all, packed as the heap's sparse_packing setting asks: the
// Alive class is the sparse one; with packing off k_gol_death_heads runs)
__global__ __launch_bounds__(1024) void k_gol_death(HeapView h, GolK p)
{
    for_each_object_packed(h, p.alive_cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        bool die = false;
        const int32_t cid = live ? farr<int32_t>(h, bid, p.a_id)[s] : 0;
        if (live && ((uint32_t)cid >= (uint32_t)(p.W * p.H) || !gol_valid(h, p.cells[cid]))) {
            raise_error(h, ERR_BADHANDLE);
            live = false;
        }
        if (live) {
            const uint32_t hc = p.cells[cid];
            const int32_t n = fref<int32_t>(h, hc, p.c_count);
            if (n != 2 && n != 3) {
                fref<uint8_t>(h, hc, p.c_state) = 0;
                die = true;
            }
        }
        wave_release_packed(h, p.alive_cls, bid, s, die, pair);
    });
}

// Alive::death as above, unpacked (sparse_packing 0), one wavefront's pass
// over one block: walked with the block-header walker, so each lane's cell
// id is loaded in the same batch as the block's header instead of after it
__device__ __forceinline__ void gol_death_block(const HeapView &h, const GolK &p, const BlockHeads<1> &hd)
{
    const uint32_t s = lane_id();
    const uint32_t bid = hd.bid[0];
    // a block of another class has no live slot: its id is not used
    const int32_t cid = farr<int32_t>(h, bid, p.a_id)[s];
    bool live = (hd.bm(0) >> s) & 1;
    uint32_t hc = 0;
    if (live && (uint32_t)cid >= (uint32_t)(p.W * p.H)) {
        raise_error(h, ERR_BADHANDLE);
        live = false;
    }
    if (live) {
        hc = p.cells[cid];
        live = gol_valid(h, hc);
    }
    bool die = false;
    if (live) {
        const int32_t n = fref<int32_t>(h, hc, p.c_count);
        if (n != 2 && n != 3) {
            fref<uint8_t>(h, hc, p.c_state) = 0;
            die = true;
        }
    }
    wave_release_own_block(h, p.alive_cls, bid, __ballot(die));
}

__global__ __launch_bounds__(1024) void k_gol_death_heads(HeapView h, GolK p)
{
    for_each_block_heads<1>(h, p.alive_cls, p.wpg, [&](const BlockHeads<1> &hd) { gol_death_block(h, p, hd); });
}

// Cell::birth - if dead with exactly three live neighbours: becomes alive and
// gets a new Alive object (one wavefront's pass over one block)
__device__ __forceinline__ void gol_birth_block(const HeapView &h, const GolK &p, const BlockHeads<1> &hd)
{
    const uint32_t s = lane_id();
    const uint32_t bid = hd.bid[0];
    // the block's fields and a view of the Alive class's active blocks,
    // issued before the header is used (a block of another class has no
    // live slot: nothing is born, nothing stored)
    const uint8_t st = farr<uint8_t>(h, bid, p.c_state)[s];
    const int32_t n = farr<int32_t>(h, bid, p.c_count)[s];
    const int32_t id = farr<int32_t>(h, bid, p.c_id)[s];
    const ActiveView view = active_view(h, p.alive_cls);
    const bool born = ((hd.bm(0) >> s) & 1) && st == 0 && n == 3;
    if (born) farr<uint8_t>(h, bid, p.c_state)[s] = 1;
    const uint32_t a = wave_allocate(h, p.alive_cls, born, &view);
    if (born && a != kNull) fref<int32_t>(h, a, p.a_id) = id;
}

__global__ __launch_bounds__(1024) void k_gol_birth(HeapView h, GolK p)
{
    for_each_block_heads<1>(h, p.cell_cls, p.wpg, [&](const BlockHeads<1> &hd) { gol_birth_block(h, p, hd); });
}

// A whole generation's Alive::death and Cell::birth in one launch: the first
// p.death_groups work-groups walk the Alive objects of the class's snapshot
// (every block of a small heap, with the iteration bitmaps that
// Cell::count's snapshot wrote, or the list and bitmaps of an enumeration
// with snapshot), the others walk the Cell blocks.  The two decide on disjoint cells (death
// on live cells whose count is not 2 or 3, birth on dead cells with count 3),
// and the snapshot keeps the objects that births create out of the death
// walk, so the result is that of the two do-alls in order.
__global__ __launch_bounds__(1024) void k_gol_death_birth(HeapView h, GolK p)
{
    if (blockIdx.x < p.death_groups)
        for_each_block_heads_in<1>(h, p.alive_cls, p.wpg, blockIdx.x, p.death_groups,
                                   [&](const BlockHeads<1> &hd) { gol_death_block(h, p, hd); });
    else
        for_each_block_heads_in<1>(h, p.cell_cls, p.wpg, blockIdx.x - p.death_groups, gridDim.x - p.death_groups,
                                   [&](const BlockHeads<1> &hd) { gol_birth_block(h, p, hd); });
}

smmo_status bind_gol(smmo_heap *h, const smmo_gol_args &a, GolK &k)
{
    if (a.cell_class >= h->schema->nclasses || a.alive_class >= h->schema->nclasses ||
        a.cell_class == a.alive_class)
        return fail(SMMO_EINVAL, "gol: bad class ids");
    if (!a.cells || a.width <= 0 || a.height <= 0 || (int64_t)a.width * a.height > 0x7FFFFFFF)
        return fail(SMMO_EINVAL, "gol: bad grid");
    k.cell_cls = a.cell_class;
    k.alive_cls = a.alive_class;
    k.cells = a.cells;
    k.W = a.width;
    k.H = a.height;
    BIND(a.cell_class, "state", SMMO_U8, 1, &k.c_state, nullptr);
    BIND(a.cell_class, "count", SMMO_I32, 1, &k.c_count, nullptr);
    BIND(a.cell_class, "cell_id", SMMO_I32, 1, &k.c_id, nullptr);
    BIND(a.alive_class, "cell_id", SMMO_I32, 1, &k.a_id, nullptr);
    return SMMO_OK;
}

// blocks per wavefront iteration of Cell::count unless set otherwise
constexpr uint32_t kGolCountGroup = 2;

template <int Which>
smmo_status launch_gol(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_gol_args a;
    memcpy(&a, args, sizeof a);
    GolK k{};
    smmo_status s = cached_bind(h, (const void *)&launch_gol<Which>, cls, a, k,
                                [&] { return bind_gol(h, a, k); });
    if (s) return s;
    k.snap = 0;
    k.death_groups = 0;
    const uint32_t want = Which == 1 ? a.alive_class : a.cell_class;
    if (cls != want) return fail(SMMO_EINVAL, "gol: method runs on a different class");
    const LaunchShape ls = method_shape(h, cls, Which == 0 ? kGolCountGroup : 0);
    k.wpg = ls.block.x / 64;
    if ((s = ensure_enumerated(h, cls, false, st, Which == 1 && packing_wanted(h, cls, ls)))) return s;
    if (Which == 0) {
        if (ls.group == 4) hipLaunchKernelGGL(k_gol_count<4>, ls.grid, ls.block, 0, st, h->v, k);
        else if (ls.group == 2) hipLaunchKernelGGL(k_gol_count<2>, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_gol_count<1>, ls.grid, ls.block, 0, st, h->v, k);
    }
    if (Which == 1) {
        if (h->cfg.sparse_packing == 0) hipLaunchKernelGGL(k_gol_death_heads, ls.grid, ls.block, 0, st, h->v, k);
        else hipLaunchKernelGGL(k_gol_death, ls.grid, ls.block, 0, st, h->v, k);
    }
    if (Which == 2) hipLaunchKernelGGL(k_gol_birth, ls.grid, ls.block, 0, st, h->v, k);
    if ((s = launched("gol kernel"))) return s;
    if (Which == 2) note_allocation(h, a.alive_class, 64ull * h->v.M);
    return SMMO_OK;
}

// gol.generation on Cell: Cell::count, Alive::death, Cell::birth in two
// launches after the Alive snapshot: the count, then death and birth
// together (k_gol_death_birth).  On a heap of at most kDirectMaxBlocks
// blocks the count itself takes the snapshot of every block and death walks
// every block; on a larger one an enumeration of the Alive class with its
// snapshot comes first and death walks that list.
smmo_status run_gol_generation(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_gol_args a;
    memcpy(&a, args, sizeof a);
    // the generation deletes Alive objects and rewrites their iteration
    // bitmaps: a snapshot of the class taken before is gone
    if (a.alive_class < h->schema->nclasses) h->snap_pending &= ~(1u << a.alive_class);
    GolK k{};
    smmo_status s = cached_bind(h, (const void *)&run_gol_generation, cls, a, k,
                                [&] { return bind_gol(h, a, k); });
    if (s) return s;
    if (cls != a.cell_class) return fail(SMMO_EINVAL, "gol: method runs on a different class");
    const bool direct = h->v.M <= kDirectMaxBlocks;
    if (!direct && (s = ensure_enumerated(h, a.alive_class, true, st, false, false))) return s;
    const LaunchShape lc = method_shape(h, cls, kGolCountGroup);
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    k.wpg = lc.block.x / 64;
    k.snap = direct ? 1u : 0u;
    k.death_groups = 0;
    if (lc.group == 4) hipLaunchKernelGGL(k_gol_count<4>, lc.grid, lc.block, 0, st, h->v, k);
    else if (lc.group == 2) hipLaunchKernelGGL(k_gol_count<2>, lc.grid, lc.block, 0, st, h->v, k);
    else hipLaunchKernelGGL(k_gol_count<1>, lc.grid, lc.block, 0, st, h->v, k);
    if ((s = launched("gol kernel"))) return s;
    // death's work-groups come first, a multiple of eight of them so that
    // the birth work-groups keep their XCD numbering
    const LaunchShape lb = method_shape(h, cls, 0);
    const uint32_t wpg = lb.block.x / 64;
    const uint64_t dblocks = direct ? h->v.M : std::max<uint64_t>(1, h->ub_blocks[a.alive_class]);
    const uint64_t dwaves = std::min<uint64_t>(dblocks, h->cfg.grid_waves ? h->cfg.grid_waves : 64ull * h->cu_count);
    const uint32_t dgroups = (uint32_t)(((dwaves + wpg - 1) / wpg + 7) / 8 * 8);
    HeapView v = h->v;
    if (direct) v.direct |= 1u << a.alive_class;
    v.snap |= 1u << a.alive_class;
    k.wpg = wpg;
    k.snap = 0;
    k.death_groups = dgroups;
    hipLaunchKernelGGL(k_gol_death_birth, dim3(dgroups + lb.grid.x), lb.block, 0, st, v, k);
    if ((s = launched("gol kernel"))) return s;
    note_allocation(h, a.alive_class, 64ull * h->v.M);
    return SMMO_OK;
}

// ============================================================= n-body =====
struct NbodyK {
    uint32_t cls;
    uint32_t o_x, o_y, o_vx, o_vy, o_fx, o_fy, o_m;
    float G, eps2, dt;
};

// Body::compute_force with device_do over all bodies (Ch.7 "nbody").  A
// work-group owns one block of 64 bodies i (one per lane in every wave);
// its four wavefronts split the other bodies j block-wise (wave w takes
// every fourth block of R), stage each j-block in LDS and read it back as
// broadcasts.  Each wave sums one j-block (64 terms) into a fresh float32
// partial and adds the partial to its running sum with Kahan compensation;
// the four running sums are combined in wave order.  The thesis leaves this
// shared-memory tiling as future work (its "Further Optimizations").
template <bool kGuard>
__global__ __launch_bounds__(256) void k_nbody_force(HeapView h, NbodyK p)
{
    __shared__ float4 tile[4][64];
    __shared__ float2 red[4][64];
    if (heap_failed(h)) return;
    const BlockList L = block_list(h, p.cls);
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t ib = xcd_logical_wg(); ib < L.r; ib += gridDim.x) {
        const uint32_t bid = L.at(ib);
        if (ald32(h.type + bid) != p.cls) continue;     // same for the whole work-group
        const uint64_t bmi = ald(h.alloc_bm + bid);
        const float xi = farr<float>(h, bid, p.o_x)[lane];
        const float yi = farr<float>(h, bid, p.o_y)[lane];
        float ax = 0.f, ay = 0.f, cx = 0.f, cy = 0.f;
        for (uint32_t j0 = 0; j0 < L.r; j0 += 4) {
            const uint32_t jt = j0 + w;
            if (jt >= L.r) break;                        // wave-uniform
            const uint32_t jb = __builtin_amdgcn_readfirstlane(L.at(jt));
            if (__builtin_amdgcn_readfirstlane(ald32(h.type + jb)) != p.cls) continue;
            const uint64_t bmj = uniform64(ald(h.alloc_bm + jb));
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if ((bmj >> lane) & 1)
                v = make_float4(farr<float>(h, jb, p.o_x)[lane], farr<float>(h, jb, p.o_y)[lane],
                                farr<float>(h, jb, p.o_m)[lane], 0.f);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            tile[w][lane] = v;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            float tx = 0.f, ty = 0.f;
#pragma unroll 8
            for (int j = 0; j < 64; ++j) {
                const float4 q = tile[w][j];
                const float dx = q.x - xi, dy = q.y - yi;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, p.eps2));
                float inv = __frsqrt_rn(r2);
                if (kGuard) inv = r2 > 0.f ? inv : 0.f;
                const float sc = q.z * inv * (inv * inv);
                tx = fmaf(dx, sc, tx);
                ty = fmaf(dy, sc, ty);
            }
            float yx = tx - cx, t = ax + yx;
            cx = (t - ax) - yx;
            ax = t;
            float yy = ty - cy;
            t = ay + yy;
            cy = (t - ay) - yy;
            ay = t;
        }
        red[w][lane] = make_float2(ax, ay);
        __syncthreads();
        if (w == 0 && ((bmi >> lane) & 1)) {
            float sx = 0.f, sy = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sx += red[k][lane].x;
                sy += red[k][lane].y;
            }
            const float gm = p.G * farr<float>(h, bid, p.o_m)[lane];
            farr<float>(h, bid, p.o_fx)[lane] = gm * sx;
            farr<float>(h, bid, p.o_fy)[lane] = gm * sy;
        }
        __syncthreads();
    }
}

// Body::update - v += f / m dt; x += v dt (velocity first)
__global__ __launch_bounds__(1024) void k_nbody_update(HeapView h, NbodyK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        if (!((bm >> s) & 1)) return;
        const float m = farr<float>(h, bid, p.o_m)[s];
        float vx = farr<float>(h, bid, p.o_vx)[s], vy = farr<float>(h, bid, p.o_vy)[s];
        vx += farr<float>(h, bid, p.o_fx)[s] / m * p.dt;
        vy += farr<float>(h, bid, p.o_fy)[s] / m * p.dt;
        farr<float>(h, bid, p.o_vx)[s] = vx;
        farr<float>(h, bid, p.o_vy)[s] = vy;
        farr<float>(h, bid, p.o_x)[s] += vx * p.dt;
        farr<float>(h, bid, p.o_y)[s] += vy * p.dt;
    });
}

smmo_status bind_nbody(smmo_heap *h, uint32_t cls, const smmo_nbody_args &a, NbodyK &k)
{
    if (!(a.eps >= 0.f) || !(a.dt == a.dt) || !(a.G == a.G)) return fail(SMMO_EINVAL, "nbody: bad parameters");
    k.cls = cls;
    BIND(cls, "pos_x", SMMO_F32, 1, &k.o_x, nullptr);
    BIND(cls, "pos_y", SMMO_F32, 1, &k.o_y, nullptr);
    BIND(cls, "vel_x", SMMO_F32, 1, &k.o_vx, nullptr);
    BIND(cls, "vel_y", SMMO_F32, 1, &k.o_vy, nullptr);
    BIND(cls, "force_x", SMMO_F32, 1, &k.o_fx, nullptr);
    BIND(cls, "force_y", SMMO_F32, 1, &k.o_fy, nullptr);
    BIND(cls, "mass", SMMO_F32, 1, &k.o_m, nullptr);
    k.G = a.G;
    k.eps2 = a.eps * a.eps;
    k.dt = a.dt;
    return SMMO_OK;
}

smmo_status nbody_force_launch(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_nbody_args a;
    memcpy(&a, args, sizeof a);
    NbodyK k;
    smmo_status s = cached_bind(h, (const void *)&nbody_force_launch, cls, a, k,
                                [&] { return bind_nbody(h, cls, a, k); });
    if (s) return s;
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, h->ub_blocks[cls]), 8192);
    if (k.eps2 > 0.f)
        hipLaunchKernelGGL(k_nbody_force<false>, dim3(grid), dim3(256), 0, st, h->v, k);
    else
        hipLaunchKernelGGL(k_nbody_force<true>, dim3(grid), dim3(256), 0, st, h->v, k);
    return launched("k_nbody_force");
}

smmo_status nbody_update_launch(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_nbody_args a;
    memcpy(&a, args, sizeof a);
    NbodyK k;
    smmo_status s = cached_bind(h, (const void *)&nbody_update_launch, cls, a, k,
                                [&] { return bind_nbody(h, cls, a, k); });
    if (s) return s;
    if ((s = ensure_enumerated(h, cls, false, st))) return s;
    hipLaunchKernelGGL(k_nbody_update, method_shape(h, cls).grid, method_shape(h, cls).block, 0, st, h->v, k);
    return launched("k_nbody_update");
}

// ======================================================= test methods =====
struct AxpyK {
    uint32_t cls, o_x;
    float a, b;
};

// packed do-all (sparse blocks two per wavefront where the heap's
// sparse_packing setting asks for it)
__global__ __launch_bounds__(1024) void k_axpy(HeapView h, AxpyK p)
{
    for_each_object_packed(h, p.cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        if (live) {
            float &x = farr<float>(h, bid, p.o_x)[s];
            x = p.a * x + p.b;
        }
    });
}

smmo_status launch_axpy(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_axpy_args a;
    memcpy(&a, args, sizeof a);
    AxpyK k{cls, 0, a.a, a.b};
    BIND(cls, "x", SMMO_F32, 1, &k.o_x, nullptr);
    const LaunchShape ls = method_shape(h, cls);
    smmo_status s = ensure_enumerated(h, cls, false, st, packing_wanted(h, cls, ls));
    if (s) return s;
    hipLaunchKernelGGL(k_axpy, ls.grid, ls.block, 0, st, h->v, k);
    return launched("k_axpy");
}

struct DestroyIfK {
    uint32_t cls, o_key;
    int32_t mod, rem;
};

__global__ __launch_bounds__(1024) void k_destroy_if(HeapView h, DestroyIfK p)
{
    for_each_object_packed(h, p.cls, false, [&](uint32_t bid, uint32_t s, bool live, bool pair) {
        bool d = false;
        if (live) {
            const int32_t key = farr<int32_t>(h, bid, p.o_key)[s];
            int32_t m = key % p.mod;
            if (m < 0) m += p.mod;
            d = m == p.rem;
        }
        wave_release_packed(h, p.cls, bid, s, d, pair);
    });
}

smmo_status launch_destroy_if(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_destroy_if_args a;
    memcpy(&a, args, sizeof a);
    if (a.mod <= 0) return fail(SMMO_EINVAL, "destroy_if: mod must be > 0");
    DestroyIfK k{cls, 0, a.mod, a.rem};
    BIND(cls, "key", SMMO_I32, 1, &k.o_key, nullptr);
    const LaunchShape ls = method_shape(h, cls);
    smmo_status s = ensure_enumerated(h, cls, false, st, packing_wanted(h, cls, ls));
    if (s) return s;
    hipLaunchKernelGGL(k_destroy_if, ls.grid, ls.block, 0, st, h->v, k);
    return launched("k_destroy_if");
}

struct SpawnK {
    uint32_t cls, target, o_key, t_key;
    int32_t mod, rem, mul, add;
    uint32_t copies, snapshot;
};

__global__ __launch_bounds__(1024) void k_spawn(HeapView h, SpawnK p)
{
    for_each_block(h, p.cls, p.snapshot != 0, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        bool sp = false;
        int32_t key = 0;
        if ((bm >> s) & 1) {
            key = farr<int32_t>(h, bid, p.o_key)[s];
            int32_t m = key % p.mod;
            if (m < 0) m += p.mod;
            sp = m == p.rem;
        }
        for (uint32_t c = 0; c < p.copies; ++c) {
            const uint32_t nh = wave_allocate(h, p.target, sp);
            if (sp && nh != kNull) fref<int32_t>(h, nh, p.t_key) = key * p.mul + p.add + (int32_t)c;
        }
    });
}

// test.transmute: the selected objects create their copies of the other
// class, then delete themselves (the replacement pattern of the thesis's
// Game of Life, Alive -> Candidate)
__global__ __launch_bounds__(1024) void k_transmute(HeapView h, SpawnK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        const uint32_t s = lane_id();
        bool sel = false;
        int32_t key = 0;
        if ((bm >> s) & 1) {
            key = farr<int32_t>(h, bid, p.o_key)[s];
            int32_t m = key % p.mod;
            if (m < 0) m += p.mod;
            sel = m == p.rem;
        }
        for (uint32_t c = 0; c < p.copies; ++c) {
            const uint32_t nh = wave_allocate(h, p.target, sel);
            if (sel && nh != kNull) fref<int32_t>(h, nh, p.t_key) = key * p.mul + p.add + (int32_t)c;
        }
        wave_release_own_block(h, p.cls, bid, __ballot(sel));
    });
}

smmo_status launch_transmute(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_spawn_args a;
    memcpy(&a, args, sizeof a);
    if (a.mod <= 0 || a.copies > 8 || a.target_class >= h->schema->nclasses || a.target_class == cls)
        return fail(SMMO_EINVAL, "transmute: bad arguments");
    SpawnK k{cls, a.target_class, 0, 0, a.mod, a.rem, a.key_mul, a.key_add, a.copies, 0u};
    BIND(cls, "key", SMMO_I32, 1, &k.o_key, nullptr);
    BIND(a.target_class, "key", SMMO_I32, 1, &k.t_key, nullptr);
    smmo_status s = ensure_enumerated(h, cls, false, st);
    if (s) return s;
    const LaunchShape ls = method_shape(h, cls);
    hipLaunchKernelGGL(k_transmute, ls.grid, ls.block, 0, st, h->v, k);
    if ((s = launched("k_transmute"))) return s;
    note_allocation(h, a.target_class, 64ull * h->v.M);
    return SMMO_OK;
}

smmo_status launch_spawn(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_spawn_args a;
    memcpy(&a, args, sizeof a);
    if (a.mod <= 0 || a.copies > 8 || a.target_class >= h->schema->nclasses)
        return fail(SMMO_EINVAL, "spawn: bad arguments");
    SpawnK k{cls, a.target_class, 0, 0, a.mod, a.rem, a.key_mul, a.key_add, a.copies,
             a.target_class == cls ? 1u : 0u};
    BIND(cls, "key", SMMO_I32, 1, &k.o_key, nullptr);
    BIND(a.target_class, "key", SMMO_I32, 1, &k.t_key, nullptr);
    smmo_status s = ensure_enumerated(h, cls, k.snapshot != 0, st);
    if (s) return s;
    hipLaunchKernelGGL(k_spawn, method_shape(h, cls).grid, method_shape(h, cls).block, 0, st, h->v, k);
    if ((s = launched("k_spawn"))) return s;
    note_allocation(h, a.target_class, 64ull * h->v.M);
    return SMMO_OK;
}

// ============================================ allocator microbenchmark =====
// Linux Scalability (Ch.8 "Raw Allocation Performance"): each worker object
// allocates n objects of the target class through the device allocator, then
// a second do-all frees them.  The objects' memory is not touched.
struct LsK {
    uint32_t cls, target, o_id, n, workers;
    uint32_t *handles;
};

__device__ __forceinline__ bool ls_worker(const HeapView &h, const LsK &p, uint32_t bid, uint64_t bm,
                                          uint32_t &id)
{
    const uint32_t s = lane_id();
    id = 0;
    if (!((bm >> s) & 1)) return false;
    id = (uint32_t)farr<int32_t>(h, bid, p.o_id)[s];
    if (id >= p.workers) {
        raise_error(h, ERR_BADHANDLE);
        return false;
    }
    return true;
}

__global__ __launch_bounds__(1024) void k_ls_alloc(HeapView h, LsK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        uint32_t id;
        const bool live = ls_worker(h, p, bid, bm, id);
        for (uint32_t i = 0; i < p.n; ++i) {
            if (__builtin_amdgcn_readfirstlane(ald32(h.ctrl + CTRL_ERR))) break;
            const uint32_t hd = wave_allocate(h, p.target, live);
            if (live) p.handles[(uint64_t)i * p.workers + id] = hd;
        }
    });
}

__global__ __launch_bounds__(1024) void k_ls_free(HeapView h, LsK p)
{
    for_each_block(h, p.cls, false, [&](uint32_t bid, uint64_t bm) {
        uint32_t id;
        const bool live = ls_worker(h, p, bid, bm, id);
        for (uint32_t i = 0; i < p.n; ++i) {
            uint32_t hd = kNull;
            bool want = false;
            if (live) {
                hd = p.handles[(uint64_t)i * p.workers + id];
                if (hd != kNull) {
                    const uint32_t b = hd >> 6;
                    want = b < h.M && ald32(h.type + b) == p.target;
                    if (!want) raise_error(h, ERR_BADHANDLE);
                }
            }
            wave_deallocate(h, p.target, hd, want);
        }
    });
}

template <int Which>
smmo_status launch_ls(smmo_heap *h, uint32_t cls, const void *args, hipStream_t st)
{
    smmo_ls_args a;
    memcpy(&a, args, sizeof a);
    if (!a.handles || a.n == 0 || a.workers == 0 || a.target_class >= h->schema->nclasses ||
        a.target_class == cls)
        return fail(SMMO_EINVAL, "alloc.ls: bad arguments");
    if ((uint64_t)a.n * a.workers > 0xFFFFFFFFull) return fail(SMMO_EINVAL, "alloc.ls: n * workers too large");
    LsK k{cls, a.target_class, 0, a.n, a.workers, a.handles};
    BIND(cls, "id", SMMO_I32, 1, &k.o_id, nullptr);
    smmo_status s = ensure_enumerated(h, cls, false, st);
    if (s) return s;
    const LaunchShape ls = method_shape(h, cls);
    if (Which == 0) hipLaunchKernelGGL(k_ls_alloc, ls.grid, ls.block, 0, st, h->v, k);
    else hipLaunchKernelGGL(k_ls_free, ls.grid, ls.block, 0, st, h->v, k);
    if ((s = launched("alloc.ls kernel"))) return s;
    if (Which == 0) note_allocation(h, a.target_class, (uint64_t)a.n * a.workers);
    return SMMO_OK;
}

} // namespace

namespace smmo {
smmo_status launch_gol_cell_count(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_gol<0>(h, c, a, s); }
smmo_status launch_gol_alive_death(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_gol<1>(h, c, a, s); }
smmo_status launch_gol_cell_birth(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_gol<2>(h, c, a, s); }
smmo_status launch_gol_generation(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return run_gol_generation(h, c, a, s); }
smmo_status launch_nbody_force(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return nbody_force_launch(h, c, a, s); }
smmo_status launch_nbody_update(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return nbody_update_launch(h, c, a, s); }
smmo_status launch_test_axpy(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_axpy(h, c, a, s); }
smmo_status launch_test_destroy_if(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_destroy_if(h, c, a, s); }
smmo_status launch_test_spawn(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_spawn(h, c, a, s); }
smmo_status launch_test_transmute(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_transmute(h, c, a, s); }
smmo_status launch_ls_alloc(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_ls<0>(h, c, a, s); }
smmo_status launch_ls_free(smmo_heap *h, uint32_t c, const void *a, hipStream_t s) { return launch_ls<1>(h, c, a, s); }
} // namespace smmo
