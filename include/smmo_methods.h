/*
 * smmo_methods.h - methods compiled into libsmmo and their argument structs.
 *
 * A C ABI cannot take device lambdas or member-function pointers, so the
 * methods that smmo_parallel_do() can run are compiled into the library and
 * named by id (smmo_method_id(name)).  Each method states the class it runs
 * on and the fields it needs by name and type; smmo_parallel_do() resolves
 * them in the class's layout and returns SMMO_EINVAL if one is missing.
 * Argument structs are passed by host pointer and size and copied at launch.
 */
#ifndef SMMO_METHODS_H
#define SMMO_METHODS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- Game of Life in SMMO form (thesis Ch.7 "gol", rule B3/S23) --------
 * Cell  {state: U8, count: I32, cell_id: I32}   one per cell, never deleted
 * Alive {cell_id: I32}                          one per live cell
 * "gol.cell_count"  on Cell : count = live cells among the 8 torus neighbours
 * "gol.alive_death" on Alive: if its cell's count is not 2 or 3, set the cell
 *                             dead and delete this Alive object
 * "gol.cell_birth"  on Cell : if dead and count == 3, set alive and create an
 *                             Alive object for the cell
 * "gol.generation"  on Cell : one whole generation, with the result of the
 *                             three do-alls above in that order: the count,
 *                             then death and birth in one launch (they
 *                             decide on disjoint cells), after the Alive
 *                             class's iteration snapshot, which keeps the
 *                             new Alive objects out of the death walk.  On a
 *                             heap of at most 8,192 blocks the count takes
 *                             the snapshot of every block; on a larger one
 *                             an enumeration of the Alive class with its
 *                             snapshot comes first (three launches).  A
 *                             snapshot of the Alive class pending from
 *                             smmo_snapshot is dropped.
 * cells[i] is the handle of the Cell with cell_id i (the thesis keeps Cell
 * pointers in a global array); the grid is width x height, index y*width+x. */
typedef struct {
    uint32_t cell_class;
    uint32_t alive_class;
    const uint32_t *cells;      /* device, width*height handles */
    int32_t width;
    int32_t height;
} smmo_gol_args;

/* ---- n-body (thesis Ch.7 "nbody") ----------------------------------------
 * Body {pos_x, pos_y, vel_x, vel_y, force_x, force_y, mass: F32}
 * "nbody.force"  : force = sum over all other bodies j (a device_do over the
 *                  class) of G m m_j (x_j - x) / (|x_j - x|^2 + eps^2)^(3/2)
 * "nbody.update" : vel += force / mass * dt; pos += vel * dt               */
typedef struct {
    float G;
    float eps;
    float dt;
    uint32_t reserved;
} smmo_nbody_args;

/* ---- spring-mass mesh (thesis Ch.7 "structure", compute steps) -----------
 * Node   {x, y, vx, vy, m: F32, adj: HANDLE x 8}
 *        adj[q] = spring handle | (1 << 31 if this node is the spring's
 *        endpoint b), SMMO_NULL for an empty slot
 * Spring {a, b: HANDLE (nodes), k, L0, fx, fy: F32, slot_a, slot_b: U8}
 *        slot_a / slot_b: index of this spring in a.adj / b.adj
 * "spring.force"       on Spring: d = x_b - x_a, l = |d|; if
 *        (l - L0) / L0 > strain_limit the spring empties its two adjacency
 *        slots and deletes itself; otherwise (fx, fy) = k (l - L0) d / l,
 *        the force on a (b receives the negative).  With
 *        SMMO_SPRING_TENSION_ONLY in flags a spring only pulls (the thesis's
 *        springs, Ch.7 "structure": Hooke's law while stretched): (fx, fy) = 0
 *        while l <= L0.
 * "spring.node_update" on Node: F = sum over occupied slots, in slot order,
 *        of +-(fx, fy); v += F / m * dt; x += v * dt.
 * "spring.link"        on Spring: writes the spring's handle into a.adj[slot_a]
 *        and (handle | 1 << 31) into b.adj[slot_b]; builds the topology after
 *        parallel_new of the nodes (adj empty) and the springs.               */
#define SMMO_SPRING_TENSION_ONLY 1u
typedef struct {
    uint32_t node_class;
    uint32_t spring_class;
    float dt;
    float strain_limit;
    uint32_t flags;              /* 0 or SMMO_SPRING_TENSION_ONLY; other bits: SMMO_EINVAL */
} smmo_spring_args;

/* ---- spring-mass mesh with partially inlined adjacency --------------------
 * The adjacency of a node is an inner array whose first K slots are inlined
 * as SOA arrays in the node's block and whose other slots live outside the
 * heap (Ch.4 sec.4.3.1 "SOA with Partial Inlining"), for meshes of
 * high-degree nodes:
 * Node   {x, y, vx, vy, m: F32, adj: HANDLE x K, more: I32, cap: I32}
 *        slots 0..cap-1 of the node: q < K in adj[q], q >= K in
 *        overflow[more + q - K]; entries as for "spring.*" (spring handle |
 *        1 << 31 if this node is the spring's endpoint b, SMMO_NULL empty)
 * Spring {a, b: HANDLE, k, L0, fx, fy: F32, slot_a, slot_b: U8}
 * "spring_pi.force", "spring_pi.node_update", "spring_pi.link": the methods
 * "spring.force", "spring.node_update" and "spring.link" (two-sided Hooke's
 * law, the float32 strain break) with this slot storage.  A slot outside
 * 0..cap-1 or an overflow index outside the array sets SMMO_EDEVICE. */
typedef struct {
    uint32_t node_class;
    uint32_t spring_class;
    float dt;
    float strain_limit;
    uint32_t *overflow;          /* device array of the out-of-line slots */
    uint64_t overflow_len;       /* its entries */
} smmo_spring_pi_args;

/* ---- reverse mode through the spring-mesh step (breaking off) ------------
 * Node   additionally {lx, ly, lvx, lvy, wx, wy: F32, id: I32}
 *        (dL/dx, dL/dv and the weighted velocity adjoint w = M^-1 mu)
 * Spring additionally {cx, cy, gk: F32}
 *        (dt K g of the current reverse step, accumulated dL/dk)
 * For L = f(x_T), a reverse step n (T-1 .. 0) from the adjoints at n+1 is
 *   mu = lv + dt lx; w = mu / m; lv = mu;                      (Node)
 *   g = w_a - w_b; u = d / l at x_n; K g = k((1 - L0/l) g + (L0/l) u (u.g));
 *   c = dt K g; gk += dt (l - L0)(u.g)                          (Spring)
 *   lx -= c at endpoint a, += c at endpoint b, in slot order    (Node)
 * "adjoint.record" on Node  : tape plane pair `slot` <- (x, y), by handle
 * "adjoint.save"   on Node  : tape planes 4*slot .. 4*slot+3 <- (x, y, vx, vy)
 * "adjoint.load"   on Node  : (x, y, vx, vy) <- those planes
 * "adjoint.seed"   on Node  : lx, ly <- seed_x[id], seed_y[id]; lvx, lvy <-
 *                             seed_vx[id], seed_vy[id] (0 if NULL)
 * "adjoint.zero"   on Spring: gk = cx = cy = 0
 * "adjoint.node"   on Node  : mode bit 0: add the springs' c terms to lx, ly;
 *                             mode bit 1: mu, w, lv as above (bit 0 first)
 * "adjoint.spring" on Spring: c and gk with positions x_n read from tape
 *                             plane pair `slot`
 * "adjoint.step_node" on Node: the node pass of the forward step (the update
 *                             of "spring.node_update" from the Spring fields
 *                             fx, fy that "spring.force" wrote); with a
 *                             non-NULL tape the new (x, y) also go to tape
 *                             plane pair `slot`, by handle (tape NULL: no
 *                             tape, tape_floats and plane unused)
 * The tape holds planes of `plane` floats (plane >= 64 * heap blocks, one
 * float per handle); tape_floats is its capacity, checked on the host.
 * seed arrays have seed_count entries, indexed by the node's id field.     */
typedef struct {
    uint32_t node_class;
    uint32_t spring_class;
    float dt;
    uint32_t mode;
    float *tape;
    uint64_t tape_floats;
    uint64_t plane;
    uint32_t slot;
    uint32_t seed_count;
    const float *seed_x;
    const float *seed_y;
    const float *seed_vx;
    const float *seed_vy;
} smmo_adjoint_args;

/* ---- test methods ---------------------------------------------------------
 * "test.axpy"      on any class with F32 field "x": x = a * x + b
 * "test.destroy_if" on any class with I32 field "key": delete this object if
 *                   key mod `mod` == `rem` (mod > 0)
 * "test.spawn"     on any class with I32 field "key": an object whose key
 *                   mod `mod` == `rem` creates `copies` objects of class
 *                   target_class (which must have an I32 field "key") with
 *                   key = key * key_mul + key_add + c, c = 0 .. copies-1.
 *                   target_class may be the running class: the new objects
 *                   are not visited by the same launch.
 * "test.transmute" on any class with I32 field "key", arguments as
 *                   "test.spawn" with a target_class other than the running
 *                   class: a selected object creates its copies and then
 *                   deletes itself, so blocks emptied by one wavefront can be
 *                   taken by another wavefront's allocations of the other
 *                   class within the same launch.                           */
typedef struct {
    float a;
    float b;
} smmo_axpy_args;

typedef struct {
    int32_t mod;
    int32_t rem;
} smmo_destroy_if_args;

typedef struct {
    uint32_t target_class;
    int32_t mod;
    int32_t rem;
    uint32_t copies;            /* 0 .. 8 */
    int32_t key_mul;
    int32_t key_add;
} smmo_spawn_args;

/* ---- allocator microbenchmark (Ch.8 "Raw Allocation Performance", the
 * Linux Scalability benchmark in SMMO form) ---------------------------------
 * "alloc.ls_alloc" on any class with I32 field "id" (0 <= id < workers): every
 *                  object allocates n objects of target_class with the device
 *                  allocator, one after another, and stores the i-th handle
 *                  at handles[i * workers + id] (SMMO_NULL once the heap is
 *                  exhausted; the device error is then set and the remaining
 *                  allocations are skipped).
 * "alloc.ls_free"  on the same class: every object deletes the n objects
 *                  named at handles[i * workers + id]; SMMO_NULL entries are
 *                  skipped, any other handle that names no object of
 *                  target_class sets the device error (bad handle).
 * target_class must differ from the running class; handles is a device array
 * of n * workers entries owned by the caller; an id outside [0, workers)
 * sets the device error (bad handle) and that object does nothing.         */
typedef struct {
    uint32_t target_class;
    uint32_t n;
    uint32_t workers;
    uint32_t reserved;
    uint32_t *handles;
} smmo_ls_args;

/* ---- wa-tor (Ch.7 "wa-tor"): fish and sharks on a W x H torus ------------
 * Classes and fields (the thesis's Agent subclasses Fish and Shark are two
 * classes here):
 *   Cell  HANDLE "agent" (a Fish handle, a Shark handle with bit 31 set, or
 *         SMMO_NULL), HANDLE "nb" x4 (neighbour cells up, right, down, left),
 *         U8 "req" x5 (requests from those neighbours; [4] = stay), I32
 *         "cell_id" (y * width + x)
 *   Fish  HANDLE "pos", HANDLE "new_pos", I32 "timer"
 *   Shark HANDLE "pos", HANDLE "new_pos", I32 "timer", I32 "energy"
 * One iteration = cell_prepare, fish_prepare, cell_decide (kind 1),
 * fish_update, cell_prepare, shark_prepare, cell_decide (kind 2),
 * shark_update, each with iteration = t.  Random choices: the splitmix64
 * output for seed and counter ((4t + phase) << 32) + cell_id, phase 0 fish
 * prepare, 1 fish decide, 2 shark prepare, 3 shark decide, taken mod the
 * number of candidates.
 * "wator.cell_link"     on Cell: nb from cell_id, with cells[i] = handle of
 *                       the Cell with cell_id i (device array of width*height)
 * "wator.link"          on Fish (kind 1) or Shark (kind 2): its cell's agent
 *                       = this object
 * "wator.cell_prepare"  on Cell: clears req
 * "wator.fish_prepare"  on Fish: timer + 1, new_pos = pos, asks a random
 *                       empty neighbour (or to stay)
 * "wator.shark_prepare" on Shark: timer + 1, energy - 1, new_pos = pos, asks
 *                       a random neighbour with a fish, else a random empty
 *                       one (or to stay)
 * "wator.cell_decide"   on Cell: grants its own agent's stay request, or one
 *                       random requesting neighbour's agent of class `kind`
 *                       (new_pos = this cell)
 * "wator.fish_update"   on Fish: moves if granted; after more than
 *                       fish_spawn iterations a moving fish leaves a new Fish
 * "wator.shark_update"  on Shark: dies (deletes itself) when energy <= 0;
 *                       else moves if granted, deletes the fish it lands on
 *                       (energy + boost), and after more than shark_spawn
 *                       iterations leaves a new Shark with energy0         */
typedef struct {
    uint32_t cell_class;
    uint32_t fish_class;
    uint32_t shark_class;
    uint32_t iteration;
    uint64_t seed;
    int32_t fish_spawn;
    int32_t shark_spawn;
    int32_t energy0;
    int32_t boost;
    uint32_t kind;
    int32_t width;
    int32_t height;
    uint32_t reserved;
    const uint32_t *cells;
} smmo_wator_args;

/* ---- generation (thesis Ch.7 "generation": Game of Life with dying cells) --
 * Cell  {state: U8 (0 empty, 1 live, 2 dying), count: I32, cell_id: I32}
 * Alive {cell_id: I32, left: I32 (dying generations left, 0 while live),
 *        is_new: U8}
 * One generation on a W x H torus = "generation.cell_count", then
 * "generation.cell_birth", then "generation.alive_update":
 * "generation.cell_count"   on Cell: count = live (state 1) neighbours.
 * "generation.cell_birth"   on Cell: an empty cell whose count is in the
 *        birth set becomes live and gets a new Alive (left 0, is_new 1).
 * "generation.alive_update" on Alive: a new object only clears is_new; a
 *        live one whose cell's count is not in the survive set starts dying
 *        (left = dying, cell state 2); a dying one counts left down and, at
 *        0, empties its cell (state 0) and deletes itself.
 * Births run before the update so that they see the generation's starting
 * states; is_new keeps the update away from this generation's births.  The
 * thesis's rule "Burst" is survive {0,2,3,5,6,7,8}, birth {3,4,6,8},
 * dying 255. */
typedef struct {
    uint32_t cell_class;
    uint32_t alive_class;
    int32_t width;
    int32_t height;
    uint32_t survive;            /* bit c: a live cell with c live neighbours stays live (c = 0..8) */
    uint32_t birth;              /* bit c: an empty cell with c live neighbours comes alive */
    int32_t dying;               /* generations a dead cell keeps blocking, >= 1 */
    uint32_t reserved;
    const uint32_t *cells;       /* W*H Cell handles, index y*W + x */
} smmo_generation_args;

/* ---- structure (thesis Ch.7 "structure": fracture of a spring mesh) -------
 * Class hierarchy (smmo_define_subclass; inherited fields first):
 * NodeBase (abstract) {x, y: F32, springs: HANDLE x 3, nspr: I32, dist: I32,
 *        id: I32}; springs[q] = spring handle | (1 << 31 if this node is the
 *        spring's p2), SMMO_NULL for an empty slot; nspr = occupied slots
 * AnchorNode     : NodeBase {}                 fixed
 * AnchorPullNode : NodeBase {vx, vy: F32}      moves at a constant velocity
 * Node           : NodeBase {vx, vy, m: F32}   moves under the spring forces
 * Spring {p1, p2: HANDLE (any NodeBase class), k, L0, maxf, fx, fy: F32,
 *        s1, s2: U8 (slot of the spring in p1 / p2), del: U8, id: I32}
 * Unlinking a spring from a node empties the node's slot and decrements
 * nspr; the unlink that takes nspr to 0 deletes the node.
 * "structure.pull"        on AnchorPullNode: x += vx dt, y += vy dt.
 * "structure.force"       on Spring: d = x_p2 - x_p1, l = |d|; stretched iff
 *        l > L0 and F = k (l - L0) (both in float32: l2 = fma(dx, dx, dy*dy),
 *        l = sqrt(l2) correctly rounded, each operation rounded); if
 *        stretched and F > maxf the spring unlinks itself from p1 and p2 and
 *        deletes itself; else (fx, fy) = k (l - L0) d / l if stretched, (0, 0)
 *        if slack: the force on p1 (p2 receives the negative).
 * "structure.node_update" on Node: F = sum over the occupied slots, in slot
 *        order, of +-(fx, fy); v += F / m dt; x += v dt.
 * "structure.bfs_init"    on NodeBase (all node classes): dist = 0 for
 *        AnchorNode objects, SMMO_STRUCTURE_FAR for the others.
 * "structure.bfs_visit"   on NodeBase: a node with dist == distance sets
 *        *flag = 1 and gives each neighbour with dist SMMO_STRUCTURE_FAR the
 *        distance distance + 1.
 * "structure.bfs_mark"    on NodeBase: a node with dist SMMO_STRUCTURE_FAR
 *        sets del on its springs.
 * "structure.bfs_delete"  on Spring: a spring with del set unlinks itself
 *        from p1 and p2 and deletes itself.
 * "structure.link"        on Spring: writes the spring's handle into
 *        p1.springs[s1] and (handle | 1 << 31) into p2.springs[s2]; builds the
 *        topology after parallel_new of the nodes (springs empty, nspr set)
 *        and the springs.
 * A do-all on NodeBase runs once per concrete node class; the methods bind
 * the node fields on nodebase_class, whose offsets every node class shares. */
#define SMMO_STRUCTURE_FAR 0x7FFFFFFF
/* Forms of smmo_structure_remove_disconnected with the same results, for
 * tests and measurements of the paths that large meshes take: the visited
 * set in device memory for every node (without it, only for the node slots
 * beyond 1,177,600), and a frontier buffer in LDS of 64 nodes instead of
 * 2,048 (the queue in device memory takes the rest). */
#define SMMO_BFS_DEVICE_VISITED 1u
#define SMMO_BFS_SMALL_FRONTIER 2u
typedef struct {
    uint32_t nodebase_class;
    uint32_t anchor_class;
    uint32_t spring_class;
    int32_t distance;            /* bfs_visit: the frontier's distance */
    float dt;                    /* pull, node_update */
    uint32_t bfs_options;        /* smmo_structure_remove_disconnected: 0, or
                                    SMMO_BFS_* bits */
    uint32_t *flag;              /* bfs_visit: device word, set to 1 when the
                                    frontier is not empty; the caller clears it */
} smmo_structure_args;

#ifdef __cplusplus
}
#endif
#endif /* SMMO_METHODS_H */
