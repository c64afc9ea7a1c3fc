/*
 * CPU oracle of SMMO execution.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow C; float64 arithmetic; array-of-structs object stores.  Only
 * the test suite, the smoke check and the bench's CPU-baseline leg load this
 * library.  It shares no code, header, table or helper with the HIP library,
 * and it never calls it.
 *
 * Semantics followed (Springer, "Memory-Efficient Object-Oriented Programming
 * on GPUs"):
 *   - Single-Method Multiple-Objects, Ch.3 sec.3.2.1 "Definition and Runtime
 *     Semantics": a parallel do-all runs a method once for every object of a
 *     class that exists when the operation starts; objects created during it
 *     are not visited; the order is unspecified; a method may delete only its
 *     own object (as its last statement) or objects of other classes.
 *   - DynaSOAr interface, Ch.5 sec.5.1.1: parallel_new constructs n objects,
 *     passing the index 0..n-1 to the constructor; device_do is a sequential
 *     loop over all objects of a class inside one method execution.
 * A do-all here takes a snapshot of the live object ids and calls the method
 * on each id in ascending order, one after the other.  Every method below
 * reads only fields that the same do-all does not write (or its own
 * object's), so this sequential loop is one valid schedule of the parallel
 * operation.  For the same reason the do-alls of the n-body and spring-mesh
 * methods, which write only their own object, may hand the snapshot to
 * several host threads (OpenMP, OMP_NUM_THREADS): any interleaving of such
 * calls gives the same result as the loop.  The one shared update among
 * them, a spring deleting itself (the free list and the break count), is
 * serialized.  Sums over other objects stay sequential loops inside one
 * call, so results do not depend on the thread count.
 *
 * Parity pins (what checks this file against something other than itself)
 * are in tests/test_oracle_*.py.  Block and slot placement is not modelled:
 * the oracle keeps live sets only, and results are compared through key
 * fields (cell index, node id, spring id).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Object store: one per class.  Objects have ids; destroyed ids are reused.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    size_t size;          /* bytes per object */
    size_t n;             /* ids handed out so far (high-water mark) */
    size_t cap;
    unsigned char *data;
    unsigned char *live;
    size_t *freelist;
    size_t nfree;
    size_t nlive;
} ostore;

static int os_init(ostore *s, size_t size, size_t cap)
{
    memset(s, 0, sizeof *s);
    s->size = size;
    s->cap = cap ? cap : 16;
    s->data = calloc(s->cap, size);
    s->live = calloc(s->cap, 1);
    s->freelist = malloc(s->cap * sizeof(size_t));
    return (s->data && s->live && s->freelist) ? 0 : -1;
}

static void os_free(ostore *s)
{
    free(s->data);
    free(s->live);
    free(s->freelist);
    memset(s, 0, sizeof *s);
}

static void *os_at(const ostore *s, size_t id) { return s->data + id * s->size; }

/* new: reuse the most recently freed id, else the next unused one */
static long long os_new(ostore *s)
{
    size_t id;
    if (s->nfree) {
        id = s->freelist[--s->nfree];
    } else {
        if (s->n == s->cap) {
            size_t nc = s->cap * 2;
            unsigned char *d = realloc(s->data, nc * s->size);
            unsigned char *l = realloc(s->live, nc);
            size_t *f = realloc(s->freelist, nc * sizeof(size_t));
            if (!d || !l || !f) return -1;
            s->data = d; s->live = l; s->freelist = f;
            memset(s->live + s->cap, 0, nc - s->cap);
            s->cap = nc;
        }
        id = s->n++;
    }
    memset(os_at(s, id), 0, s->size);
    s->live[id] = 1;
    s->nlive++;
    return (long long)id;
}

/* destroy: deleting a dead object is a usage error; report it */
static int os_destroy(ostore *s, size_t id)
{
    if (id >= s->n || !s->live[id]) return -1;
    s->live[id] = 0;
    s->freelist[s->nfree++] = id;
    s->nlive--;
    return 0;
}

/* the set of objects a do-all visits: those alive when it starts */
static size_t os_snapshot(const ostore *s, size_t *ids)
{
    size_t k = 0;
    for (size_t i = 0; i < s->n; i++)
        if (s->live[i]) ids[k++] = i;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Game of Life in SMMO form (thesis Ch.7 "gol"; rule B3/S23 as stated       */
/* there: a live cell stays alive with two or three live neighbours, a dead  */
/* cell becomes alive with exactly three).                                   */
/*                                                                           */
/* Classes: Cell {state u8, count i32, cell_id i32}, one per grid cell and   */
/* never destroyed; Alive {cell_id i32}, one per live cell, created on birth */
/* and destroyed on death (the thesis attaches an Alive agent to every live  */
/* cell).  Grid: W x H torus, cell index y*W + x.                             */
/* One generation = three do-alls:                                            */
/*   Cell::count  - number of live cells among the 8 torus neighbours        */
/*   Alive::death - if its cell's count is not 2 or 3: cell state = 0,        */
/*                  delete this                                               */
/*   Cell::birth  - if state == 0 and count == 3: state = 1, new Alive        */
/* ------------------------------------------------------------------------ */
typedef struct { uint8_t state; int32_t count; int32_t cell_id; } gol_cell;
typedef struct { int32_t cell_id; } gol_alive;

typedef struct {
    int W, H;
    ostore cell, alive;
    size_t *cells;   /* cell index -> Cell object id (the thesis's Cell::cells array) */
    size_t *snap;
    int err;
} gol_world;

static void gol_cell_count(gol_world *w, gol_cell *c)
{
    int x = c->cell_id % w->W, y = c->cell_id / w->W, n = 0;
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            if (!dx && !dy) continue;
            int nx = (x + dx + w->W) % w->W, ny = (y + dy + w->H) % w->H;
            const gol_cell *o = os_at(&w->cell, w->cells[(size_t)ny * w->W + nx]);
            n += o->state;
        }
    c->count = n;
}

static void gol_alive_death(gol_world *w, size_t self)
{
    gol_alive *a = os_at(&w->alive, self);
    gol_cell *c = os_at(&w->cell, w->cells[a->cell_id]);
    if (c->count != 2 && c->count != 3) {
        c->state = 0;
        if (os_destroy(&w->alive, self)) w->err = 1;   /* last statement: delete this */
    }
}

static void gol_cell_birth(gol_world *w, gol_cell *c)
{
    if (c->state == 0 && c->count == 3) {
        c->state = 1;
        long long id = os_new(&w->alive);
        if (id < 0) { w->err = 2; return; }
        ((gol_alive *)os_at(&w->alive, (size_t)id))->cell_id = c->cell_id;
    }
}

void *orc_gol_create(int W, int H, const uint8_t *init)
{
    if (W <= 0 || H <= 0) return NULL;
    gol_world *w = calloc(1, sizeof *w);
    size_t nc = (size_t)W * H;
    w->W = W; w->H = H;
    w->cells = malloc(nc * sizeof(size_t));
    w->snap = malloc(nc * sizeof(size_t));
    if (os_init(&w->cell, sizeof(gol_cell), nc) || os_init(&w->alive, sizeof(gol_alive), nc)) return NULL;
    /* parallel_new<Cell>(W*H): constructor(index) */
    for (size_t i = 0; i < nc; i++) {
        long long id = os_new(&w->cell);
        gol_cell *c = os_at(&w->cell, (size_t)id);
        c->state = init[i] ? 1 : 0;
        c->count = 0;
        c->cell_id = (int32_t)i;
        w->cells[i] = (size_t)id;
    }
    /* one Alive per initially live cell, in ascending cell index */
    for (size_t i = 0; i < nc; i++)
        if (init[i]) {
            long long id = os_new(&w->alive);
            ((gol_alive *)os_at(&w->alive, (size_t)id))->cell_id = (int32_t)i;
        }
    return w;
}

int orc_gol_step(void *wp, int steps)
{
    gol_world *w = wp;
    for (int s = 0; s < steps; s++) {
        size_t k = os_snapshot(&w->cell, w->snap);
        for (size_t i = 0; i < k; i++) gol_cell_count(w, os_at(&w->cell, w->snap[i]));
        k = os_snapshot(&w->alive, w->snap);
        for (size_t i = 0; i < k; i++) gol_alive_death(w, w->snap[i]);
        k = os_snapshot(&w->cell, w->snap);
        for (size_t i = 0; i < k; i++) gol_cell_birth(w, os_at(&w->cell, w->snap[i]));
    }
    return w->err;
}

/* state and count per cell index; sorted cell indices of the live Alive objects */
long long orc_gol_read(void *wp, uint8_t *state, int32_t *count, int32_t *alive_cells)
{
    gol_world *w = wp;
    size_t nc = (size_t)w->W * w->H;
    for (size_t i = 0; i < nc; i++) {
        const gol_cell *c = os_at(&w->cell, w->cells[i]);
        if (state) state[i] = c->state;
        if (count) count[i] = c->count;
    }
    long long n = 0;
    if (alive_cells) {
        /* counting sort over cell indices gives the canonical (ascending) set */
        unsigned char *mark = calloc(nc, 1);
        for (size_t i = 0; i < w->alive.n; i++)
            if (w->alive.live[i]) {
                int32_t cid = ((gol_alive *)os_at(&w->alive, i))->cell_id;
                if (mark[cid]) w->err = 3;   /* two Alive objects on one cell */
                mark[cid] = 1;
            }
        for (size_t i = 0; i < nc; i++)
            if (mark[i]) alive_cells[n++] = (int32_t)i;
        free(mark);
    } else {
        n = (long long)w->alive.nlive;
    }
    return n;
}

int orc_gol_error(void *wp) { return ((gol_world *)wp)->err; }

void orc_gol_free(void *wp)
{
    gol_world *w = wp;
    if (!w) return;
    os_free(&w->cell);
    os_free(&w->alive);
    free(w->cells);
    free(w->snap);
    free(w);
}

/* ------------------------------------------------------------------------ */
/* n-body (thesis Ch.7 "nbody"): class Body {x, y, vx, vy, fx, fy, m}.        */
/*   Body::compute_force: f = 0, then a device_do over all bodies adds the   */
/*     gravitational pull of every other body j:                             */
/*       f += G m_i m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2)            */
/*     (Newton's law F = G m1 m2 / r^2 along the connecting line; eps is a    */
/*     Plummer softening length, eps = 0 gives the thesis's unsoftened law).  */
/*   Body::update: v += f / m * dt, then x += v * dt with the new v (the      */
/*     thesis's time step: velocity first, position from the new velocity).  */
/* The thesis's wall bounce is not part of this method set.                  */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, vx, vy, fx, fy, m, sx, sy; } nb_body;

/* device_do<Body>(&Body::apply_force) seen from body `self` */
static void nb_force(const ostore *st, const size_t *all, size_t nall, size_t self,
                     double G, double eps2)
{
    nb_body *b = os_at(st, self);
    double fx = 0, fy = 0, sx = 0, sy = 0;
    for (size_t t = 0; t < nall; t++) {
        if (all[t] == self) continue;   /* the thesis skips other == this */
        const nb_body *o = os_at(st, all[t]);
        double dx = o->x - b->x, dy = o->y - b->y;
        double r2 = dx * dx + dy * dy + eps2;
        double c = G * b->m * o->m / (r2 * sqrt(r2));
        fx += c * dx;
        fy += c * dy;
        sx += fabs(c * dx);
        sy += fabs(c * dy);
    }
    b->fx = fx; b->fy = fy; b->sx = sx; b->sy = sy;
}

static void nb_update(nb_body *b, double dt)
{
    b->vx += b->fx / b->m * dt;
    b->vy += b->fy / b->m * dt;
    b->x += b->vx * dt;
    b->y += b->vy * dt;
}

/*
 * `steps` iterations of {compute_force, update} on n bodies, arrays updated in
 * place.  sfx/sfy (may be NULL) receive sum_j |term_ij| per component of the
 * last force evaluation: the conditioning scale used by the parity tolerance.
 */
int orc_nbody_steps(long long n, double *x, double *y, double *vx, double *vy,
                    double *fx, double *fy, const double *m, double G, double eps,
                    double dt, int steps, double *sfx, double *sfy)
{
    ostore st;
    if (n < 0 || os_init(&st, sizeof(nb_body), (size_t)(n ? n : 1))) return -1;
    size_t *snap = malloc((size_t)(n ? n : 1) * sizeof(size_t));
    for (long long i = 0; i < n; i++) {   /* parallel_new<Body>(n) */
        nb_body *b = os_at(&st, (size_t)os_new(&st));
        b->x = x[i]; b->y = y[i]; b->vx = vx[i]; b->vy = vy[i]; b->m = m[i];
    }
    for (int s = 0; s < steps; s++) {
        size_t k = os_snapshot(&st, snap);
#pragma omp parallel for schedule(dynamic, 64)
        for (size_t i = 0; i < k; i++) nb_force(&st, snap, k, snap[i], G, eps * eps);
        k = os_snapshot(&st, snap);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < k; i++) nb_update(os_at(&st, snap[i]), dt);
    }
    for (long long i = 0; i < n; i++) {   /* ids equal the construction index */
        const nb_body *b = os_at(&st, (size_t)i);
        x[i] = b->x; y[i] = b->y; vx[i] = b->vx; vy[i] = b->vy;
        if (fx) fx[i] = b->fx;
        if (fy) fy[i] = b->fy;
        if (sfx) sfx[i] = b->sx;
        if (sfy) sfy[i] = b->sy;
    }
    free(snap);
    os_free(&st);
    return 0;
}

/* Body::update alone, from given forces (arrays updated in place) */
int orc_nbody_update(long long n, double *x, double *y, double *vx, double *vy,
                     const double *fx, const double *fy, const double *m, double dt)
{
    ostore st;
    if (n < 0 || os_init(&st, sizeof(nb_body), (size_t)(n ? n : 1))) return -1;
    size_t *snap = malloc((size_t)(n ? n : 1) * sizeof(size_t));
    for (long long i = 0; i < n; i++) {
        nb_body *b = os_at(&st, (size_t)os_new(&st));
        b->x = x[i]; b->y = y[i]; b->vx = vx[i]; b->vy = vy[i];
        b->fx = fx[i]; b->fy = fy[i]; b->m = m[i];
    }
    size_t k = os_snapshot(&st, snap);
    for (size_t i = 0; i < k; i++) nb_update(os_at(&st, snap[i]), dt);
    for (long long i = 0; i < n; i++) {
        const nb_body *b = os_at(&st, (size_t)i);
        x[i] = b->x; y[i] = b->y; vx[i] = b->vx; vy[i] = b->vy;
    }
    free(snap);
    os_free(&st);
    return 0;
}

/* compute_force for selected bodies only (the device_do of those bodies) */
int orc_nbody_force_at(long long n, const double *x, const double *y, const double *m,
                       double G, double eps, const long long *idx, long long nidx,
                       double *fx, double *fy, double *sfx, double *sfy)
{
    ostore st;
    if (n < 0 || os_init(&st, sizeof(nb_body), (size_t)(n ? n : 1))) return -1;
    size_t *snap = malloc((size_t)(n ? n : 1) * sizeof(size_t));
    for (long long i = 0; i < n; i++) {
        nb_body *b = os_at(&st, (size_t)os_new(&st));
        b->x = x[i]; b->y = y[i]; b->m = m[i];
    }
    size_t k = os_snapshot(&st, snap);
    for (long long t = 0; t < nidx; t++) {
        if (idx[t] < 0 || idx[t] >= n) { free(snap); os_free(&st); return -2; }
        nb_force(&st, snap, k, (size_t)idx[t], G, eps * eps);
        const nb_body *b = os_at(&st, (size_t)idx[t]);
        fx[t] = b->fx; fy[t] = b->fy;
        if (sfx) sfx[t] = b->sx;
        if (sfy) sfy[t] = b->sy;
    }
    free(snap);
    os_free(&st);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Spring-mass mesh (thesis Ch.7 "structure", its compute steps):           */
/*   Spring::compute_force - Hooke's law F = k * dx on the spring's two     */
/*     endpoints; a spring stretched past its limit breaks: it unlinks      */
/*     itself from both nodes and deletes itself.                            */
/*   Node::update - sum the forces of the attached springs, then            */
/*     accelerate and move as in nbody (v += F/m dt, x += v dt).             */
/* Readings where the thesis leaves the details open (listed in the design   */
/* notes): the spring pulls and pushes (two-sided Hooke's law on the length  */
/* change l - L0), the force on endpoint a is k (l - L0) d / l with          */
/* d = x_b - x_a and the force on b is its negative; a spring breaks when    */
/* its strain (l - L0) / L0 exceeds a threshold, and it then exerts no force */
/* in that step.  Both decisions (break; for tension-only springs, which    */
/* give no force while l <= L0, slack) are taken in float64 from the state  */
/* as given: the plain definition of the rule, in no particular float32     */
/* operation order.                                                          */
/* Ties.  A float32 implementation fed the same float32 state computes the  */
/* strain with an error of a few units in the last place (dx, dy rounded,   */
/* the square, the sum and the root rounded, l - L0 exact near the limit,   */
/* the quotient rounded: about 4.2 * 2^-24 = 2.5e-7 near strain 0.3).  A     */
/* spring whose float64 strain lies within SP_TIE_STRAIN of the threshold is */
/* a tie: either decision is correct.  A caller may fix the decision of     */
/* such springs for the first step of a call (tie[s] = 0 keep, 1 break,     */
/* -1 decide); fixing one outside the band is an error.  Slack ties need no */
/* such care: there the force k (l - L0) is within rounding of zero.        */
/* Nodes keep up to 8 spring slots; a break empties the two slots (the       */
/* spring remembers its slot index in each node); Node::update sums the      */
/* occupied slots in slot order.                                             */
/* ------------------------------------------------------------------------ */
#define SP_DEG 8

typedef struct {
    double x, y, vx, vy, m;
    long long adj[SP_DEG];     /* spring object id, -1 = empty slot */
    uint8_t adjb[SP_DEG];      /* 1 if this node is the spring's endpoint b */
    double svx, svy, sx, sy;   /* conditioning scales of the last update */
} sp_node;

typedef struct {
    long long a, b;            /* node object ids */
    double k, L0, fx, fy, sf;
    int32_t sa, sb;            /* slot of this spring in a.adj / b.adj */
} sp_spring;

typedef struct {
    ostore node, spring;
    size_t *snap;
    double thresh;
    int tension_only;
    double dt;
    long long nbroken;
    int err;
    const int8_t *tie;         /* fixed decisions of ties in the first step, or NULL */
    double *strain;            /* strain of each spring at its last force pass, or NULL */
    int first;                 /* 1 during the first step of the call */
} sp_world;

/* half-width of the tie band around the break threshold, in strain (see above) */
#define SP_TIE_STRAIN 1e-6

/* the break decision of one spring in float64: strain (l - L0) / L0 above
 * the threshold; *strain receives the strain */
static int sp_breaks(double xa, double ya, double xb, double yb, double L0, double thresh, double *strain)
{
    const double dx = xb - xa, dy = yb - ya;
    const double l = sqrt(dx * dx + dy * dy);
    *strain = (l - L0) / L0;
    return *strain > thresh;
}

/* the decision of spring `sid` with strain `strain`: the rule, or the fixed
 * decision of a tie; -1 if a fixed decision lies outside the tie band */
static int sp_decide(const int8_t *tie, long long sid, double strain, double thresh, int rule)
{
    if (!tie || tie[sid] < 0) return rule;
    if (!(fabs(strain - thresh) <= SP_TIE_STRAIN)) return -1;
    return tie[sid] != 0;
}

static void sp_spring_force(sp_world *w, size_t self)
{
    sp_spring *s = os_at(&w->spring, self);
    sp_node *a = os_at(&w->node, (size_t)s->a);
    sp_node *b = os_at(&w->node, (size_t)s->b);
    double strain;
    int brk = sp_breaks(a->x, a->y, b->x, b->y, s->L0, w->thresh, &strain);
    if (w->strain) w->strain[self] = strain;
    brk = sp_decide(w->first ? w->tie : NULL, (long long)self, strain, w->thresh, brk);
    if (brk < 0) {
#pragma omp atomic write
        w->err = 8;
        return;
    }
    if (brk) {
        if (a->adj[s->sa] != (long long)self || b->adj[s->sb] != (long long)self) {
#pragma omp atomic write
            w->err = 4;
        }
        a->adj[s->sa] = -1;     /* the two slots are this spring's own */
        b->adj[s->sb] = -1;
        s->fx = s->fy = s->sf = 0;
        int bad;
#pragma omp critical(sp_delete)
        {
            w->nbroken++;
            bad = os_destroy(&w->spring, self);   /* last statement: delete this */
        }
        if (bad) {
#pragma omp atomic write
            w->err = 5;
        }
        return;
    }
    double dx = b->x - a->x, dy = b->y - a->y;
    double l = sqrt(dx * dx + dy * dy);
    /* scale of the float32 rounding error of f: the terms k l and k L0 of
     * k (l - L0) in magnitude (also for a slack spring, whose decision is
     * within that error of the other one at a tie) */
    s->sf = s->k * (l + s->L0);
    if (w->tension_only && !(l > s->L0)) {
        s->fx = s->fy = 0;     /* slack: a tension-only spring does not push */
        return;
    }
    double c = s->k * (l - s->L0) / l;
    s->fx = c * dx;
    s->fy = c * dy;
}

static void sp_node_update(sp_world *w, sp_node *n)
{
    double Fx = 0, Fy = 0, SF = 0;
    for (int q = 0; q < SP_DEG; q++) {
        if (n->adj[q] < 0) continue;
        const sp_spring *s = os_at(&w->spring, (size_t)n->adj[q]);
        double sg = n->adjb[q] ? -1.0 : 1.0;
        Fx += sg * s->fx;
        Fy += sg * s->fy;
        SF += s->sf;
    }
    n->svx = fabs(n->vx) + w->dt * SF / n->m;
    n->svy = fabs(n->vy) + w->dt * SF / n->m;
    n->sx = fabs(n->x) + w->dt * n->svx;
    n->sy = fabs(n->y) + w->dt * n->svy;
    n->vx += Fx / n->m * w->dt;
    n->vy += Fy / n->m * w->dt;
    n->x += n->vx * w->dt;
    n->y += n->vy * w->dt;
}

/*
 * `steps` iterations of {Spring::compute_force, Node::update} on a mesh given
 * by arrays indexed by node id (N) and spring id (S); updated in place.
 *   adj:   N*8 spring ids (-1 empty), adjb: N*8 endpoint-b flags
 *   alive: S flags (0 = spring already broken; such ids must not be in adj)
 * Optional outputs (NULL to skip), all of the last step:
 *   sf (S)               scale of each spring force
 *   svx, svy, sx, sy (N) scales of the node velocity and position updates
 *   strain (S)           strain of each spring at its last force pass
 *                        (entries of springs dead at the start untouched)
 * tension_only: springs give no force while l <= L0 (see above).
 * tie (S, or NULL): fixed decisions of ties in the first step (see above).
 * Returns the number of springs broken, or a negative error code (-18: a
 * fixed decision outside the tie band).
 */
long long orc_spring_steps(long long N, double *x, double *y, double *vx, double *vy,
                           const double *m, int32_t *adj, const uint8_t *adjb,
                           long long S, const int32_t *a, const int32_t *b,
                           const double *k, const double *L0,
                           const int32_t *slot_a, const int32_t *slot_b,
                           uint8_t *alive, double *fx, double *fy,
                           double dt, double thresh, int steps,
                           double *sf, double *svx, double *svy, double *sx, double *sy,
                           int tension_only, const int8_t *tie, double *strain)
{
    sp_world w;
    memset(&w, 0, sizeof w);
    w.dt = dt;
    w.thresh = thresh;
    w.tension_only = tension_only != 0;
    w.tie = tie;
    w.strain = strain;
    if (N < 0 || S < 0) return -1;
    if (os_init(&w.node, sizeof(sp_node), (size_t)(N ? N : 1)) ||
        os_init(&w.spring, sizeof(sp_spring), (size_t)(S ? S : 1))) return -1;
    size_t big = (size_t)(N > S ? N : S);
    w.snap = malloc((big ? big : 1) * sizeof(size_t));
    for (long long i = 0; i < N; i++) {      /* parallel_new<Node>(N) */
        sp_node *n = os_at(&w.node, (size_t)os_new(&w.node));
        n->x = x[i]; n->y = y[i]; n->vx = vx[i]; n->vy = vy[i]; n->m = m[i];
        for (int q = 0; q < SP_DEG; q++) {
            n->adj[q] = adj[i * SP_DEG + q];
            n->adjb[q] = adjb[i * SP_DEG + q];
        }
    }
    for (long long i = 0; i < S; i++) {      /* parallel_new<Spring>(S) */
        sp_spring *s = os_at(&w.spring, (size_t)os_new(&w.spring));
        s->a = a[i]; s->b = b[i]; s->k = k[i]; s->L0 = L0[i];
        s->sa = slot_a[i]; s->sb = slot_b[i];
        s->fx = fx ? fx[i] : 0; s->fy = fy ? fy[i] : 0;
    }
    for (long long i = 0; i < S; i++)        /* springs broken before this call */
        if (!alive[i]) os_destroy(&w.spring, (size_t)i);
    for (long long i = 0; i < N; i++)
        for (int q = 0; q < SP_DEG; q++) {
            long long sid = adj[i * SP_DEG + q];
            if (sid >= S || (sid >= 0 && !alive[sid])) w.err = 6;
        }
    for (int st = 0; st < steps && !w.err; st++) {
        w.first = st == 0;
        size_t kk = os_snapshot(&w.spring, w.snap);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < kk; i++) sp_spring_force(&w, w.snap[i]);
        kk = os_snapshot(&w.node, w.snap);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < kk; i++) sp_node_update(&w, os_at(&w.node, w.snap[i]));
    }
    for (long long i = 0; i < N; i++) {
        const sp_node *n = os_at(&w.node, (size_t)i);
        x[i] = n->x; y[i] = n->y; vx[i] = n->vx; vy[i] = n->vy;
        for (int q = 0; q < SP_DEG; q++) adj[i * SP_DEG + q] = (int32_t)n->adj[q];
        if (svx) svx[i] = n->svx;
        if (svy) svy[i] = n->svy;
        if (sx) sx[i] = n->sx;
        if (sy) sy[i] = n->sy;
    }
    for (long long i = 0; i < S; i++) {
        const sp_spring *s = os_at(&w.spring, (size_t)i);
        alive[i] = w.spring.live[i];
        if (fx) fx[i] = s->fx;
        if (fy) fy[i] = s->fy;
        if (sf) sf[i] = s->sf;
    }
    free(w.snap);
    os_free(&w.node);
    os_free(&w.spring);
    return w.err ? -(long long)w.err - 10 : w.nbroken;
}

/* the break decision alone, for tests of its edge cases; *strain (or NULL)
 * receives the strain */
int orc_spring_breaks(double xa, double ya, double xb, double yb, double L0, double thresh, double *strain)
{
    double e;
    const int r = sp_breaks(xa, ya, xb, yb, L0, thresh, &e);
    if (strain) *strain = e;
    return r;
}

/* threads the OpenMP do-alls use (reported with CPU timings) */
int orc_threads(void) { return omp_get_max_threads(); }

/* sets them (n >= 1): the tests compare results at one and several threads */
void orc_set_threads(int n) { omp_set_num_threads(n < 1 ? 1 : n); }

/* half-width of the tie band (for the tests that count ties) */
double orc_spring_tie_band(void) { return SP_TIE_STRAIN; }

/* ------------------------------------------------------------------------ */
/* Differentiable spring mesh (reverse mode through the compute steps above,  */
/* topology fixed: no spring breaks).  Not in the thesis; it is the reverse   */
/* of one step                                                               */
/*   v_{n+1} = v_n + dt M^-1 f(x_n; k),   x_{n+1} = x_n + dt v_{n+1}          */
/* for the loss L = 1/2 sum_i |x_i(T) - xhat_i|^2.  With adjoints lx = dL/dx, */
/* lv = dL/dv, starting from lx_T = x_T - xhat, lv_T = 0, step n (T-1 .. 0):  */
/*   mu = lv_{n+1} + dt lx_{n+1};  w = M^-1 mu;  lv_n = mu                     */
/*   per spring (a, b) at positions x_n: d = x_b - x_a, l = |d|, u = d / l,   */
/*     g = w_a - w_b,  K g = k ((1 - L0/l) g + (L0/l) u (u . g)),             */
/*     dL/dk += dt (l - L0) (u . g);   lx_a -= dt K g;  lx_b += dt K g        */
/*   lx_n = lx_{n+1} + (those spring terms)                                  */
/* Positions x_n are recomputed per segment from (x, v) checkpoints taken    */
/* every `every` steps of the forward pass.  Each reverse step is three       */
/* do-alls: Node (mu, w, lv), Spring (K g, dL/dk), Node (sum of spring terms  */
/* in slot order).                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lx, ly, lvx, lvy, wx, wy;
} adj_node;

typedef struct {
    double cx, cy, gk;
    double agk;     /* sum over the reverse steps of dt |g| (see below) */
} adj_spring;

static void adj_node_mu(sp_world *w, adj_node *an, const sp_node *n)
{
    (void)w;
    double mux = an->lvx + w->dt * an->lx, muy = an->lvy + w->dt * an->ly;
    an->wx = mux / n->m;
    an->wy = muy / n->m;
    an->lvx = mux;
    an->lvy = muy;
}

static void adj_spring_jg(sp_world *w, size_t self, const double *px, const double *py,
                          const adj_node *an, adj_spring *as)
{
    const sp_spring *s = os_at(&w->spring, self);
    double dx = px[s->b] - px[s->a], dy = py[s->b] - py[s->a];
    double l = sqrt(dx * dx + dy * dy);
    double ux = dx / l, uy = dy / l;
    double gx = an[s->a].wx - an[s->b].wx, gy = an[s->a].wy - an[s->b].wy;
    double ug = ux * gx + uy * gy;
    double kgx = s->k * ((1.0 - s->L0 / l) * gx + (s->L0 / l) * ux * ug);
    double kgy = s->k * ((1.0 - s->L0 / l) * gy + (s->L0 / l) * uy * ug);
    as[self].cx = w->dt * kgx;
    as[self].cy = w->dt * kgy;
    as[self].gk += w->dt * (l - s->L0) * ug;
    as[self].agk += w->dt * sqrt(gx * gx + gy * gy);
}

static void adj_node_sum(sp_world *w, size_t self, adj_node *an, const adj_spring *as)
{
    const sp_node *n = os_at(&w->node, self);
    for (int q = 0; q < SP_DEG; q++) {
        if (n->adj[q] < 0) continue;
        const adj_spring *c = &as[n->adj[q]];
        if (n->adjb[q]) { an[self].lx += c->cx; an[self].ly += c->cy; }
        else { an[self].lx -= c->cx; an[self].ly -= c->cy; }
    }
}

/*
 * Forward T steps from (x, y, vx, vy) with breaking off, then the reverse
 * sweep.  Outputs (NULL to skip): gk (S), gvx, gvy, gx, gy (N) = dL/dk,
 * dL/dv0, dL/dx0; xT, yT (N) final positions; *loss; agk (S) = the sum over
 * the reverse steps of dt |g|, which bounds the factor dt |u . g| with which
 * each step's stretch l - L0 enters dL/dk (an error e in every stretch moves
 * dL/dk by at most e agk).  `every` = checkpoint interval (1..T).  Returns 0,
 * or a negative error code.
 */
int orc_spring_adjoint(long long N, const double *x, const double *y, const double *vx,
                       const double *vy, const double *m, const int32_t *adj, const uint8_t *adjb,
                       long long S, const int32_t *a, const int32_t *b, const double *k,
                       const double *L0, const int32_t *slot_a, const int32_t *slot_b,
                       const double *xhat, const double *yhat, double dt, int T, int every,
                       double *gk, double *gvx, double *gvy, double *gx, double *gy,
                       double *xT, double *yT, double *loss, double *agk)
{
    if (N < 0 || S < 0 || T < 0 || every < 1) return -1;
    sp_world w;
    memset(&w, 0, sizeof w);
    w.dt = dt;
    w.thresh = INFINITY;
    if (os_init(&w.node, sizeof(sp_node), (size_t)(N ? N : 1)) ||
        os_init(&w.spring, sizeof(sp_spring), (size_t)(S ? S : 1))) return -1;
    size_t big = (size_t)(N > S ? N : S);
    w.snap = malloc((big ? big : 1) * sizeof(size_t));
    for (long long i = 0; i < N; i++) {
        sp_node *n = os_at(&w.node, (size_t)os_new(&w.node));
        n->x = x[i]; n->y = y[i]; n->vx = vx[i]; n->vy = vy[i]; n->m = m[i];
        for (int q = 0; q < SP_DEG; q++) { n->adj[q] = adj[i * SP_DEG + q]; n->adjb[q] = adjb[i * SP_DEG + q]; }
    }
    for (long long i = 0; i < S; i++) {
        sp_spring *s = os_at(&w.spring, (size_t)os_new(&w.spring));
        s->a = a[i]; s->b = b[i]; s->k = k[i]; s->L0 = L0[i]; s->sa = slot_a[i]; s->sb = slot_b[i];
    }
    int nck = (T + every - 1) / every + 1;
    double *ck = malloc((size_t)nck * 4 * (size_t)(N ? N : 1) * sizeof(double));
    double *tx = malloc((size_t)every * (size_t)(N ? N : 1) * sizeof(double));
    double *ty = malloc((size_t)every * (size_t)(N ? N : 1) * sizeof(double));
    adj_node *an = calloc((size_t)(N ? N : 1), sizeof(adj_node));
    adj_spring *as = calloc((size_t)(S ? S : 1), sizeof(adj_spring));
    if (!ck || !tx || !ty || !an || !as) return -1;

    /* forward, checkpoint (x, v) at steps 0, every, 2 every, ... */
    for (int n = 0; n < T; n++) {
        if (n % every == 0) {
            double *c = ck + (size_t)(n / every) * 4 * N;
            for (long long i = 0; i < N; i++) {
                const sp_node *p = os_at(&w.node, (size_t)i);
                c[i] = p->x; c[N + i] = p->y; c[2 * N + i] = p->vx; c[3 * N + i] = p->vy;
            }
        }
        size_t kk = os_snapshot(&w.spring, w.snap);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < kk; i++) sp_spring_force(&w, w.snap[i]);
        kk = os_snapshot(&w.node, w.snap);
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < kk; i++) sp_node_update(&w, os_at(&w.node, w.snap[i]));
    }
    if (w.nbroken) w.err = 7;
    double L = 0;
    for (long long i = 0; i < N; i++) {
        const sp_node *p = os_at(&w.node, (size_t)i);
        double ex = p->x - xhat[i], ey = p->y - yhat[i];
        L += 0.5 * (ex * ex + ey * ey);
        an[i].lx = ex; an[i].ly = ey; an[i].lvx = 0; an[i].lvy = 0;
        if (xT) xT[i] = p->x;
        if (yT) yT[i] = p->y;
    }
    /* reverse, segment by segment */
    for (int seg = (T - 1) / every; seg >= 0 && T > 0; seg--) {
        int n0 = seg * every, n1 = n0 + every < T ? n0 + every : T;
        const double *c = ck + (size_t)seg * 4 * N;
        for (long long i = 0; i < N; i++) {
            sp_node *p = os_at(&w.node, (size_t)i);
            p->x = c[i]; p->y = c[N + i]; p->vx = c[2 * N + i]; p->vy = c[3 * N + i];
        }
        for (int n = n0; n < n1; n++) {       /* recompute the segment's positions */
            double *px = tx + (size_t)(n - n0) * N, *py = ty + (size_t)(n - n0) * N;
            for (long long i = 0; i < N; i++) {
                const sp_node *p = os_at(&w.node, (size_t)i);
                px[i] = p->x; py[i] = p->y;
            }
            size_t kk = os_snapshot(&w.spring, w.snap);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < kk; i++) sp_spring_force(&w, w.snap[i]);
            kk = os_snapshot(&w.node, w.snap);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < kk; i++) sp_node_update(&w, os_at(&w.node, w.snap[i]));
        }
        for (int n = n1 - 1; n >= n0; n--) {
            const double *px = tx + (size_t)(n - n0) * N, *py = ty + (size_t)(n - n0) * N;
            size_t kk = os_snapshot(&w.node, w.snap);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < kk; i++) adj_node_mu(&w, &an[w.snap[i]], os_at(&w.node, w.snap[i]));
            kk = os_snapshot(&w.spring, w.snap);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < kk; i++) adj_spring_jg(&w, w.snap[i], px, py, an, as);
            kk = os_snapshot(&w.node, w.snap);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < kk; i++) adj_node_sum(&w, w.snap[i], an, as);
        }
    }
    for (long long i = 0; i < S; i++) {
        if (gk) gk[i] = as[i].gk;
        if (agk) agk[i] = as[i].agk;
    }
    for (long long i = 0; i < N; i++) {
        if (gvx) gvx[i] = an[i].lvx;
        if (gvy) gvy[i] = an[i].lvy;
        if (gx) gx[i] = an[i].lx;
        if (gy) gy[i] = an[i].ly;
    }
    if (loss) *loss = L;
    free(ck); free(tx); free(ty); free(an); free(as); free(w.snap);
    os_free(&w.node);
    os_free(&w.spring);
    return w.err ? -(int)w.err - 10 : 0;
}

/*
 * One reverse step in isolation (the three do-alls above), from given
 * positions x_n and adjoints (lx, ly, lvx, lvy) = at step n+1; they are
 * replaced by the adjoints at step n.  gk receives this step's contribution
 * to dL/dk.  Conditioning scales of the float32 rounding error (NULL to
 * skip): sgk (S) = dt (l + L0) |g|; slx, sly (N) = |lx| + sum over the
 * node's springs of dt k (1 + 2 L0/l) |g|; slv (N) = |lv| + dt |lx|.
 */
int orc_spring_adjoint_step(long long N, const double *px, const double *py, const double *m,
                            const int32_t *adj, const uint8_t *adjb, long long S, const int32_t *a,
                            const int32_t *b, const double *k, const double *L0, double dt,
                            double *lx, double *ly, double *lvx, double *lvy, double *gk,
                            double *sgk, double *slx, double *sly, double *slvx, double *slvy)
{
    if (N < 0 || S < 0) return -1;
    sp_world w;
    memset(&w, 0, sizeof w);
    w.dt = dt;
    if (os_init(&w.node, sizeof(sp_node), (size_t)(N ? N : 1)) ||
        os_init(&w.spring, sizeof(sp_spring), (size_t)(S ? S : 1))) return -1;
    size_t big = (size_t)(N > S ? N : S);
    w.snap = malloc((big ? big : 1) * sizeof(size_t));
    adj_node *an = calloc((size_t)(N ? N : 1), sizeof(adj_node));
    adj_spring *as = calloc((size_t)(S ? S : 1), sizeof(adj_spring));
    for (long long i = 0; i < N; i++) {
        sp_node *n = os_at(&w.node, (size_t)os_new(&w.node));
        n->x = px[i]; n->y = py[i]; n->m = m[i];
        for (int q = 0; q < SP_DEG; q++) { n->adj[q] = adj[i * SP_DEG + q]; n->adjb[q] = adjb[i * SP_DEG + q]; }
        an[i].lx = lx[i]; an[i].ly = ly[i]; an[i].lvx = lvx[i]; an[i].lvy = lvy[i];
    }
    for (long long i = 0; i < S; i++) {
        sp_spring *s = os_at(&w.spring, (size_t)os_new(&w.spring));
        s->a = a[i]; s->b = b[i]; s->k = k[i]; s->L0 = L0[i];
    }
    if (slvx) for (long long i = 0; i < N; i++) {
        slvx[i] = fabs(lvx[i]) + dt * fabs(lx[i]);
        slvy[i] = fabs(lvy[i]) + dt * fabs(ly[i]);
    }
    size_t kk = os_snapshot(&w.node, w.snap);
    for (size_t i = 0; i < kk; i++) adj_node_mu(&w, &an[w.snap[i]], os_at(&w.node, w.snap[i]));
    kk = os_snapshot(&w.spring, w.snap);
    for (size_t i = 0; i < kk; i++) adj_spring_jg(&w, w.snap[i], px, py, an, as);
    if (slx) {
        for (long long i = 0; i < N; i++) { slx[i] = fabs(an[i].lx); sly[i] = fabs(an[i].ly); }
        for (long long i = 0; i < S; i++) {
            const sp_spring *s = os_at(&w.spring, (size_t)i);
            double dx = px[s->b] - px[s->a], dy = py[s->b] - py[s->a];
            double l = sqrt(dx * dx + dy * dy);
            double g = hypot(an[s->a].wx - an[s->b].wx, an[s->a].wy - an[s->b].wy);
            double sc = dt * s->k * (1.0 + 2.0 * s->L0 / l) * g;
            slx[s->a] += sc; sly[s->a] += sc; slx[s->b] += sc; sly[s->b] += sc;
            if (sgk) sgk[i] = dt * (l + s->L0) * g;
        }
    }
    kk = os_snapshot(&w.node, w.snap);
    for (size_t i = 0; i < kk; i++) adj_node_sum(&w, w.snap[i], an, as);
    for (long long i = 0; i < N; i++) { lx[i] = an[i].lx; ly[i] = an[i].ly; lvx[i] = an[i].lvx; lvy[i] = an[i].lvy; }
    for (long long i = 0; i < S; i++) gk[i] = as[i].gk;
    free(an); free(as); free(w.snap);
    os_free(&w.node);
    os_free(&w.spring);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* wa-tor (thesis Ch.7 "wa-tor"): fish and sharks on a W x H torus of cells. */
/*                                                                          */
/* Classes (Fish and Shark stand for the thesis's Agent subclasses):         */
/*   Cell  {agent, kind (0 empty, 1 fish, 2 shark), request[5], cell_id,     */
/*          neighbours[4]: up, right, down, left}                            */
/*   Fish  {position, new_position, spawn_timer}                             */
/*   Shark {position, new_position, spawn_timer, energy}                     */
/* One iteration t is eight do-alls, in the thesis's order:                  */
/*   Cell::prepare, Fish::prepare, Cell::decide, Fish::update,              */
/*   Cell::prepare, Shark::prepare, Cell::decide, Shark::update.            */
/* Random choices are uniform picks among candidates: r mod (number of       */
/* candidates), where r is the splitmix64 output (Steele, Lea and Flood,    */
/* OOPSLA 2014) for counter (stream << 32) + cell index, with stream = 4t +  */
/* phase (0 fish prepare, 1 fish decide, 2 shark prepare, 3 shark decide),  */
/* always drawn for the cell whose method runs or on which the agent sits.  */
/* Parameters the thesis leaves open (spawn thresholds, energies) are inputs.*/
/* ------------------------------------------------------------------------ */
typedef struct {
    long long agent;      /* object id in the fish or shark store, -1 = none */
    uint8_t kind;
    uint8_t request[5];
    int32_t cell_id;
    size_t nb[4];
} wt_cell;
typedef struct { size_t pos, new_pos; int32_t spawn_timer; } wt_fish;
typedef struct { size_t pos, new_pos; int32_t spawn_timer, energy; } wt_shark;

typedef struct {
    int W, H;
    uint64_t seed;
    int32_t fish_spawn, shark_spawn, energy0, boost;
    long long t;
    ostore cell, fish, shark;
    size_t *cells;   /* cell index -> Cell object id */
    size_t *snap;
    size_t snap_cap;
    int err;
} wt_world;

static uint64_t wt_rand(uint64_t seed, uint64_t stream, uint64_t idx)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((stream << 32) + idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static wt_cell *wt_c(wt_world *w, size_t id) { return os_at(&w->cell, id); }

static size_t wt_snapshot(wt_world *w, ostore *s)
{
    if (s->n > w->snap_cap) {
        size_t *p = realloc(w->snap, s->n * sizeof(size_t));
        if (!p) { w->err = 2; return 0; }
        w->snap = p;
        w->snap_cap = s->n;
    }
    return os_snapshot(s, w->snap);
}

/* Cell::prepare: no requests yet */
static void wt_cell_prepare(wt_cell *c) { memset(c->request, 0, sizeof c->request); }

/* An agent on cell c asks to enter one neighbour: among the neighbours whose
 * kind is `want` (tried first) or, if none and `fallback` >= 0, of kind
 * `fallback`, one uniformly at random; with no candidate it asks to stay. */
static void wt_request(wt_world *w, wt_cell *c, int want, int fallback, uint64_t stream)
{
    int cand[4], n = 0;
    for (int i = 0; i < 4; i++)
        if (wt_c(w, c->nb[i])->kind == want) cand[n++] = i;
    if (n == 0 && fallback >= 0)
        for (int i = 0; i < 4; i++)
            if (wt_c(w, c->nb[i])->kind == fallback) cand[n++] = i;
    if (n == 0) {
        c->request[4] = 1;
        return;
    }
    int sel = cand[wt_rand(w->seed, stream, (uint64_t)c->cell_id) % (uint64_t)n];
    wt_c(w, c->nb[sel])->request[(sel + 2) % 4] = 1;
}

/* Fish::prepare: older by one iteration; ask for a random empty neighbour */
static void wt_fish_prepare(wt_world *w, wt_fish *f)
{
    f->spawn_timer++;
    f->new_pos = f->pos;
    wt_request(w, wt_c(w, f->pos), 0, -1, (uint64_t)(4 * w->t + 0));
}

/* Shark::prepare: older and hungrier by one iteration; ask for a random
 * neighbour with a fish, else a random empty one */
static void wt_shark_prepare(wt_world *w, wt_shark *s)
{
    s->spawn_timer++;
    s->energy--;
    s->new_pos = s->pos;
    wt_request(w, wt_c(w, s->pos), 1, 0, (uint64_t)(4 * w->t + 2));
}

/* Cell::decide: the cell's own agent stays if it asked to; otherwise one of
 * the requesting neighbours' agents (of kind `kind`), picked at random, is
 * told to move here */
static void wt_cell_decide(wt_world *w, size_t self, int kind, uint64_t stream)
{
    wt_cell *c = wt_c(w, self);
    if (c->request[4]) {
        if (kind == 1) ((wt_fish *)os_at(&w->fish, (size_t)c->agent))->new_pos = self;
        else ((wt_shark *)os_at(&w->shark, (size_t)c->agent))->new_pos = self;
        return;
    }
    int cand[4], n = 0;
    for (int i = 0; i < 4; i++)
        if (c->request[i]) cand[n++] = i;
    if (n == 0) return;
    int sel = cand[wt_rand(w->seed, stream, (uint64_t)c->cell_id) % (uint64_t)n];
    wt_cell *o = wt_c(w, c->nb[sel]);
    if (o->kind != kind || o->agent < 0) { w->err = 3; return; }
    if (kind == 1) ((wt_fish *)os_at(&w->fish, (size_t)o->agent))->new_pos = self;
    else ((wt_shark *)os_at(&w->shark, (size_t)o->agent))->new_pos = self;
}

static void wt_set(wt_cell *c, int kind, long long agent)
{
    c->kind = (uint8_t)kind;
    c->agent = agent;
}

/* Fish::update: move if granted; a fish that moves after more than
 * fish_spawn iterations leaves a new fish behind */
static void wt_fish_update(wt_world *w, size_t self)
{
    wt_fish *f = os_at(&w->fish, self);
    if (f->new_pos == f->pos) return;
    size_t old = f->pos;
    f->pos = f->new_pos;
    wt_set(wt_c(w, f->pos), 1, (long long)self);
    if (f->spawn_timer > w->fish_spawn) {
        long long id = os_new(&w->fish);
        if (id < 0) { w->err = 2; return; }
        f = os_at(&w->fish, self);          /* the store may have moved */
        wt_fish *nf = os_at(&w->fish, (size_t)id);
        nf->pos = nf->new_pos = old;
        nf->spawn_timer = 0;
        wt_set(wt_c(w, old), 1, id);
        f->spawn_timer = 0;
    } else {
        wt_set(wt_c(w, old), 0, -1);
    }
}

/* Shark::update: a shark without energy dies where it is; otherwise it moves
 * if granted, eating the fish on the target cell (energy + boost), and
 * leaves a new shark (energy0) behind after more than shark_spawn
 * iterations */
static void wt_shark_update(wt_world *w, size_t self)
{
    wt_shark *s = os_at(&w->shark, self);
    if (s->energy <= 0) {
        wt_set(wt_c(w, s->pos), 0, -1);
        if (os_destroy(&w->shark, self)) w->err = 1;    /* last statement: delete this */
        return;
    }
    if (s->new_pos == s->pos) return;
    size_t old = s->pos;
    wt_cell *tgt = wt_c(w, s->new_pos);
    if (tgt->kind == 1) {
        if (os_destroy(&w->fish, (size_t)tgt->agent)) w->err = 1;
        s->energy += w->boost;
    } else if (tgt->kind != 0) {
        w->err = 4;
        return;
    }
    s->pos = s->new_pos;
    wt_set(tgt, 2, (long long)self);
    if (s->spawn_timer > w->shark_spawn) {
        long long id = os_new(&w->shark);
        if (id < 0) { w->err = 2; return; }
        s = os_at(&w->shark, self);
        wt_shark *ns = os_at(&w->shark, (size_t)id);
        ns->pos = ns->new_pos = old;
        ns->spawn_timer = 0;
        ns->energy = w->energy0;
        wt_set(wt_c(w, old), 2, id);
        s->spawn_timer = 0;
    } else {
        wt_set(wt_c(w, old), 0, -1);
    }
}

/* kind[i] (0/1/2), timer[i] and energy[i] per cell index give the initial
 * agents; params = {fish_spawn, shark_spawn, energy0, boost} */
void *orc_wator_create(int W, int H, uint64_t seed, const int32_t *params, const uint8_t *kind,
                       const int32_t *timer, const int32_t *energy)
{
    if (W <= 0 || H <= 0) return NULL;
    wt_world *w = calloc(1, sizeof *w);
    size_t nc = (size_t)W * H;
    w->W = W; w->H = H; w->seed = seed;
    w->fish_spawn = params[0]; w->shark_spawn = params[1]; w->energy0 = params[2]; w->boost = params[3];
    w->cells = malloc(nc * sizeof(size_t));
    if (os_init(&w->cell, sizeof(wt_cell), nc) || os_init(&w->fish, sizeof(wt_fish), nc) ||
        os_init(&w->shark, sizeof(wt_shark), nc) || !w->cells)
        return NULL;
    for (size_t i = 0; i < nc; i++) {
        long long id = os_new(&w->cell);
        wt_cell *c = wt_c(w, (size_t)id);
        c->cell_id = (int32_t)i;
        c->agent = -1;
        w->cells[i] = (size_t)id;
    }
    for (size_t i = 0; i < nc; i++) {
        int x = (int)(i % W), y = (int)(i / W);
        wt_cell *c = wt_c(w, w->cells[i]);
        c->nb[0] = w->cells[(size_t)((y - 1 + H) % H) * W + x];
        c->nb[1] = w->cells[(size_t)y * W + (x + 1) % W];
        c->nb[2] = w->cells[(size_t)((y + 1) % H) * W + x];
        c->nb[3] = w->cells[(size_t)y * W + (x - 1 + W) % W];
    }
    for (size_t i = 0; i < nc; i++) {
        wt_cell *c = wt_c(w, w->cells[i]);
        if (kind[i] == 1) {
            long long id = os_new(&w->fish);
            wt_fish *f = os_at(&w->fish, (size_t)id);
            f->pos = f->new_pos = w->cells[i];
            f->spawn_timer = timer[i];
            wt_set(c, 1, id);
        }
    }
    for (size_t i = 0; i < nc; i++) {
        wt_cell *c = wt_c(w, w->cells[i]);
        if (kind[i] == 2) {
            long long id = os_new(&w->shark);
            wt_shark *s = os_at(&w->shark, (size_t)id);
            s->pos = s->new_pos = w->cells[i];
            s->spawn_timer = timer[i];
            s->energy = energy[i];
            wt_set(c, 2, id);
        }
    }
    return w;
}

int orc_wator_step(void *wp, int iterations)
{
    wt_world *w = wp;
    for (int it = 0; it < iterations && !w->err; it++) {
        size_t k = wt_snapshot(w, &w->cell);
        for (size_t i = 0; i < k; i++) wt_cell_prepare(wt_c(w, w->snap[i]));
        k = wt_snapshot(w, &w->fish);
        for (size_t i = 0; i < k; i++) wt_fish_prepare(w, os_at(&w->fish, w->snap[i]));
        k = wt_snapshot(w, &w->cell);
        for (size_t i = 0; i < k; i++) wt_cell_decide(w, w->snap[i], 1, (uint64_t)(4 * w->t + 1));
        k = wt_snapshot(w, &w->fish);
        for (size_t i = 0; i < k; i++) wt_fish_update(w, w->snap[i]);
        k = wt_snapshot(w, &w->cell);
        for (size_t i = 0; i < k; i++) wt_cell_prepare(wt_c(w, w->snap[i]));
        k = wt_snapshot(w, &w->shark);
        for (size_t i = 0; i < k; i++) wt_shark_prepare(w, os_at(&w->shark, w->snap[i]));
        k = wt_snapshot(w, &w->cell);
        for (size_t i = 0; i < k; i++) wt_cell_decide(w, w->snap[i], 2, (uint64_t)(4 * w->t + 3));
        k = wt_snapshot(w, &w->shark);
        for (size_t i = 0; i < k; i++) wt_shark_update(w, w->snap[i]);
        w->t++;
    }
    return w->err;
}

/* per cell index: kind, spawn timer and energy of its agent (0 where none);
 * counts[0..1] = live fish, live sharks.  Checks that cells and agents agree. */
int orc_wator_read(void *wp, uint8_t *kind, int32_t *timer, int32_t *energy, long long *counts)
{
    wt_world *w = wp;
    size_t nc = (size_t)w->W * w->H;
    for (size_t i = 0; i < nc; i++) {
        const wt_cell *c = wt_c(w, w->cells[i]);
        kind[i] = c->kind;
        timer[i] = 0;
        energy[i] = 0;
        if (c->kind == 1) {
            const wt_fish *f = os_at(&w->fish, (size_t)c->agent);
            if (!w->fish.live[c->agent] || f->pos != w->cells[i]) w->err = 5;
            timer[i] = f->spawn_timer;
        } else if (c->kind == 2) {
            const wt_shark *s = os_at(&w->shark, (size_t)c->agent);
            if (!w->shark.live[c->agent] || s->pos != w->cells[i]) w->err = 5;
            timer[i] = s->spawn_timer;
            energy[i] = s->energy;
        }
    }
    counts[0] = (long long)w->fish.nlive;
    counts[1] = (long long)w->shark.nlive;
    return w->err;
}

void orc_wator_free(void *wp)
{
    wt_world *w = wp;
    if (!w) return;
    os_free(&w->cell);
    os_free(&w->fish);
    os_free(&w->shark);
    free(w->cells);
    free(w->snap);
    free(w);
}

/* ------------------------------------------------------------------------ */
/* structure (thesis Ch.7 "structure": the fracture FEM).  Classes:          */
/*   NodeBase (abstract): position, up to three spring slots, the number of */
/*     occupied slots, the BFS distance;                                     */
/*   AnchorNode: fixed; AnchorPullNode: moves at a constant velocity;        */
/*   Node: moves under the spring forces (velocity, mass);                   */
/*   Spring: its two endpoint nodes, stiffness k, rest length L0, the force  */
/*     limit, the force of the last compute step, a delete flag.             */
/* One iteration: pull the pull nodes; compute steps, each Spring::force     */
/* then Node::update; remove the nodes no longer connected to an anchor     */
/* node (BFS from the anchor nodes) with their springs.                      */
/* Readings (listed in the design notes): a spring pulls only while          */
/* stretched (Hooke's law on the elongation l - L0 > 0); it breaks when that */
/* force k (l - L0) exceeds its limit, and then unlinks itself from both     */
/* endpoints and is deleted; a node whose last spring is unlinked is deleted */
/* (the unlink decrements its spring count, and the unlink that takes it to  */
/* zero deletes the node).  The force is stored on the spring as a vector,   */
/* (fx, fy) = k (l - L0) d / l with d = x_p2 - x_p1 acting on p1 (p2 gets    */
/* the negative), so that Node::update reads no other node.  The stretch    */
/* (l > L0) and break (k (l - L0) > limit) decisions are taken in float64   */
/* from the state as given, like those of the mesh springs.  A spring whose  */
/* float64 force lies within ST_TIE_REL k (l + L0) of its limit is a tie (a  */
/* float32 evaluation of k (l - L0) errs by at most about 5 * 2^-24 of that */
/* scale); the caller may fix its decision (tie[s] = 0 keep, 1 break).      */
/* State arrays (node id i, spring id s; ids are canonical, alive flags      */
/* mark the live objects):                                                   */
/*   ntype[i] 0 anchor, 1 pull, 2 node; nalive[i]; x, y, vx, vy, m;          */
/*   slot[3i+q] spring id or -1, isp2[3i+q] 1 if node i is the spring's p2;  */
/*   nspr[i] occupied slots; dist[i] BFS distance                            */
/*   p1[s], p2[s], k, L0, maxf, s1[s], s2[s] (slot in p1 / p2), salive[s],   */
/*   fx, fy, sdel[s]                                                         */
/* ------------------------------------------------------------------------ */
#define ST_ANCHOR 0
#define ST_PULL 1
#define ST_NODE 2
#define ST_MAXDIST 0x7FFFFFFF
#define ST_TIE_REL 1e-6

/* Node::remove_spring: empty the slot; the unlink that removes the last
 * spring deletes the node */
static int st_unlink(long long node, int q, long long sid, int32_t *slot, int32_t *nspr, uint8_t *nalive)
{
    if (!nalive[node] || slot[3 * node + q] != sid || nspr[node] <= 0) return 7;
    slot[3 * node + q] = -1;
    if (--nspr[node] == 0) nalive[node] = 0;
    return 0;
}

/* AnchorPullNode::pull on every pull node */
int orc_structure_pull(long long N, const int32_t *ntype, const uint8_t *nalive, double *x, double *y,
                       const double *vx, const double *vy, double dt)
{
    for (long long i = 0; i < N; i++)
        if (nalive[i] && ntype[i] == ST_PULL) {
            x[i] += vx[i] * dt;
            y[i] += vy[i] * dt;
        }
    return 0;
}

/* One compute step: Spring::force over the live springs, then Node::update
 * over the live Nodes.  sf (S) and svx, svy, sx, sy (N), optional, receive
 * the conditioning scales as for the mesh springs; F (S), optional, the
 * float64 force k (l - L0) of each live spring; tie (S), optional, fixed
 * decisions of ties (see above).  Returns the number of springs broken, or a
 * negative error code (-18: a fixed decision outside the tie band). */
long long orc_structure_step(long long N, const int32_t *ntype, uint8_t *nalive, double *x, double *y,
                             double *vx, double *vy, const double *m, int32_t *slot, const uint8_t *isp2,
                             int32_t *nspr, long long S, const int32_t *p1, const int32_t *p2,
                             const double *k, const double *L0, const double *maxf, const int32_t *s1,
                             const int32_t *s2, uint8_t *salive, double *fx, double *fy, double dt,
                             double *sf, double *svx, double *svy, double *sx, double *sy,
                             const int8_t *tie, double *F)
{
    long long nbroken = 0;
    uint8_t *snap = malloc((size_t)(S ? S : 1));
    if (!snap) return -1;
    memcpy(snap, salive, (size_t)S);
    for (long long s = 0; s < S; s++) {            /* Spring::force over the snapshot */
        if (!snap[s]) continue;
        const long long a = p1[s], b = p2[s];
        if (a < 0 || a >= N || b < 0 || b >= N || !nalive[a] || !nalive[b]) { free(snap); return -12; }
        const double dx = x[b] - x[a], dy = y[b] - y[a];
        const double l = sqrt(dx * dx + dy * dy);
        const double Fs = k[s] * (l - L0[s]);
        const int stretched = l > L0[s];
        if (F) F[s] = Fs;
        int brk = stretched && Fs > maxf[s];
        if (tie && tie[s] >= 0) {
            if (!(fabs(Fs - maxf[s]) <= ST_TIE_REL * k[s] * (l + L0[s]))) {
                free(snap);
                return -18;
            }
            brk = tie[s] != 0;
        }
        if (brk) {
            if (st_unlink(a, s1[s], s, slot, nspr, nalive) || st_unlink(b, s2[s], s, slot, nspr, nalive)) {
                free(snap);
                return -17;
            }
            salive[s] = 0;
            fx[s] = fy[s] = 0;
            if (sf) sf[s] = 0;
            nbroken++;
            continue;
        }
        /* the scale also for a slack spring: at a stretch tie its force is
         * within that rounding of zero either way */
        if (sf) sf[s] = k[s] * (l + L0[s]);
        if (!stretched) {
            fx[s] = fy[s] = 0;
            continue;
        }
        const double c = k[s] * (l - L0[s]) / l;
        fx[s] = c * dx;
        fy[s] = c * dy;
    }
    free(snap);
    for (long long i = 0; i < N; i++) {            /* Node::update over the live Nodes */
        if (!nalive[i] || ntype[i] != ST_NODE) continue;
        double Fx = 0, Fy = 0, SF = 0;
        for (int q = 0; q < 3; q++) {
            const long long s = slot[3 * i + q];
            if (s < 0) continue;
            if (s >= S || !salive[s]) return -13;
            const double sg = isp2[3 * i + q] ? -1.0 : 1.0;
            Fx += sg * fx[s];
            Fy += sg * fy[s];
            if (sf) SF += sf[s];
        }
        const double svxi = fabs(vx[i]) + dt * SF / m[i], svyi = fabs(vy[i]) + dt * SF / m[i];
        if (svx) svx[i] = svxi;
        if (svy) svy[i] = svyi;
        if (sx) sx[i] = fabs(x[i]) + dt * svxi;
        if (sy) sy[i] = fabs(y[i]) + dt * svyi;
        vx[i] += Fx / m[i] * dt;
        vy[i] += Fy / m[i] * dt;
        x[i] += vx[i] * dt;
        y[i] += vy[i] * dt;
    }
    return nbroken;
}

/* Removal of disconnected nodes: distance 0 at the anchor nodes and "infinite"
 * elsewhere; BFS levels while the frontier is not empty (the frontier of
 * level d is the set of nodes at distance d; each gives its unvisited
 * neighbours distance d + 1); every node left unvisited flags its springs;
 * every flagged spring unlinks itself from both endpoints (deleting nodes
 * whose last spring it was) and is deleted.  *levels receives the number of
 * visit passes (the last one finds an empty frontier).  Returns the number of
 * springs deleted, or a negative error code. */
long long orc_structure_bfs(long long N, const int32_t *ntype, uint8_t *nalive, int32_t *slot,
                            const uint8_t *isp2, int32_t *nspr, int32_t *dist, long long S,
                            const int32_t *p1, const int32_t *p2, const int32_t *s1, const int32_t *s2,
                            uint8_t *salive, uint8_t *sdel, int *levels)
{
    for (long long i = 0; i < N; i++)
        if (nalive[i]) dist[i] = ntype[i] == ST_ANCHOR ? 0 : ST_MAXDIST;
    int lv = 0;
    for (int d = 0;; d++) {
        int cont = 0;
        lv++;
        for (long long i = 0; i < N; i++) {
            if (!nalive[i] || dist[i] != d) continue;
            cont = 1;
            for (int q = 0; q < 3; q++) {
                const long long s = slot[3 * i + q];
                if (s < 0) continue;
                if (s >= S || !salive[s]) return -14;
                const long long o = isp2[3 * i + q] ? p1[s] : p2[s];
                if (o < 0 || o >= N || !nalive[o]) return -15;
                if (dist[o] == ST_MAXDIST) dist[o] = d + 1;
            }
        }
        if (!cont || d == ST_MAXDIST - 1) break;
    }
    *levels = lv;
    for (long long i = 0; i < N; i++)
        if (nalive[i] && dist[i] == ST_MAXDIST)
            for (int q = 0; q < 3; q++)
                if (slot[3 * i + q] >= 0) sdel[slot[3 * i + q]] = 1;
    long long ndel = 0;
    for (long long s = 0; s < S; s++) {
        if (!salive[s] || !sdel[s]) continue;
        if (st_unlink(p1[s], s1[s], s, slot, nspr, nalive) || st_unlink(p2[s], s2[s], s, slot, nspr, nalive))
            return -16;
        salive[s] = 0;
        ndel++;
    }
    return ndel;
}

/* ------------------------------------------------------------------------ */
/* generation (thesis Ch.7 "generation"): a generational cellular automaton, */
/* Game of Life extended by dying cells.  The thesis's rule is "Burst"       */
/* (0235678/3468/255): a live cell survives with a live-neighbour count in   */
/* the survive set S, otherwise it dies but keeps blocking its cell for D    */
/* more generations; an empty cell comes alive with a count in the birth set */
/* B.  Dying cells are not live neighbours and cannot be born into.  The     */
/* result is fully defined per cell, so this is that definition, on a W x H  */
/* torus (as the Game of Life here):                                         */
/*   count = live (state 1) cells among the 8 neighbours at generation t;    */
/*   state 0: -> 1 if count in B, else 0;                                    */
/*   state 1: -> 1 if count in S, else dying with D generations left;        */
/*   dying with r left: r - 1 left, and empty (0) once none is left.         */
/* state[i] (0 empty, 1 live, 2 dying) and left[i] (generations of dying     */
/* left, 0 unless dying) are updated in place; S and B are bit masks over    */
/* the counts 0..8.  Returns 0, or -1 for bad arguments.                     */
/* ------------------------------------------------------------------------ */
int orc_generation_steps(int W, int H, uint8_t *state, int32_t *left, uint32_t S, uint32_t B, int32_t D,
                         int steps)
{
    if (W <= 0 || H <= 0 || D < 1) return -1;
    const size_t n = (size_t)W * (size_t)H;
    uint8_t *ns = malloc(n);
    int32_t *nl = malloc(n * sizeof(int32_t));
    if (!ns || !nl) {
        free(ns);
        free(nl);
        return -1;
    }
    for (int st = 0; st < steps; st++) {
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                int count = 0;
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        if (!dx && !dy) continue;
                        const int xx = ((x + dx) % W + W) % W, yy = ((y + dy) % H + H) % H;
                        count += state[(size_t)yy * W + xx] == 1;
                    }
                const size_t i = (size_t)y * W + x;
                if (state[i] == 0) {
                    ns[i] = (B >> count) & 1;
                    nl[i] = 0;
                } else if (state[i] == 1) {
                    const int live = (S >> count) & 1;
                    ns[i] = live ? 1 : 2;
                    nl[i] = live ? 0 : D;
                } else {
                    nl[i] = left[i] - 1;
                    ns[i] = nl[i] > 0 ? 2 : 0;
                }
            }
        memcpy(state, ns, n);
        memcpy(left, nl, n * sizeof(int32_t));
    }
    free(ns);
    free(nl);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The spring-mass mesh above with node degree up to D (any D >= 1): the    */
/* same two steps and decisions, adjacency N*D spring ids (-1 empty) summed  */
/* in slot order.  It serves meshes whose nodes exceed the 8 slots of        */
/* orc_spring_steps (hubs), whose adjacency the GPU stores partly inlined    */
/* (Ch.4 sec.4.3.1 "SOA with Partial Inlining").  Arguments and results as   */
/* orc_spring_steps (two-sided springs).                                     */
/* ------------------------------------------------------------------------ */
long long orc_spring_steps_deg(long long N, int D, double *x, double *y, double *vx, double *vy,
                               const double *m, int32_t *adj, const uint8_t *adjb,
                               long long S, const int32_t *a, const int32_t *b,
                               const double *k, const double *L0,
                               const int32_t *slot_a, const int32_t *slot_b,
                               uint8_t *alive, double *fx, double *fy,
                               double dt, double thresh, int steps,
                               double *sf, double *svx, double *svy, double *sx, double *sy,
                               const int8_t *tie, double *strain)
{
    if (N < 0 || S < 0 || D < 1) return -1;
    double *f_x = malloc((size_t)(S ? S : 1) * sizeof(double));
    double *f_y = malloc((size_t)(S ? S : 1) * sizeof(double));
    double *s_f = malloc((size_t)(S ? S : 1) * sizeof(double));
    uint8_t *snap = malloc((size_t)(S ? S : 1));
    if (!f_x || !f_y || !s_f || !snap) {
        free(f_x); free(f_y); free(s_f); free(snap);
        return -1;
    }
    long long err = 0, nbroken = 0;
    for (long long s = 0; s < S; s++) {
        f_x[s] = fx ? fx[s] : 0;
        f_y[s] = fy ? fy[s] : 0;
        s_f[s] = 0;
    }
    for (long long i = 0; i < N && !err; i++)
        for (int q = 0; q < D; q++) {
            const long long sid = adj[i * D + q];
            if (sid >= S || (sid >= 0 && !alive[sid])) err = 6;
        }
    for (int st = 0; st < steps && !err; st++) {
        memcpy(snap, alive, (size_t)S);
        for (long long s = 0; s < S; s++) {           /* Spring::compute_force */
            if (!snap[s]) continue;
            const long long ia = a[s], ib = b[s];
            double e;
            int brk = sp_breaks(x[ia], y[ia], x[ib], y[ib], L0[s], thresh, &e);
            if (strain) strain[s] = e;
            brk = sp_decide(st == 0 ? tie : NULL, s, e, thresh, brk);
            if (brk < 0) {
                err = 8;
                break;
            }
            if (brk) {
                if (adj[ia * D + slot_a[s]] != s || adj[ib * D + slot_b[s]] != s) err = 4;
                adj[ia * D + slot_a[s]] = -1;
                adj[ib * D + slot_b[s]] = -1;
                f_x[s] = f_y[s] = s_f[s] = 0;
                alive[s] = 0;
                nbroken++;
                continue;
            }
            const double dx = x[ib] - x[ia], dy = y[ib] - y[ia];
            const double l = sqrt(dx * dx + dy * dy);
            const double c = k[s] * (l - L0[s]) / l;
            f_x[s] = c * dx;
            f_y[s] = c * dy;
            s_f[s] = k[s] * (l + L0[s]);
        }
        for (long long i = 0; i < N; i++) {           /* Node::update */
            double Fx = 0, Fy = 0, SF = 0;
            for (int q = 0; q < D; q++) {
                const long long s = adj[i * D + q];
                if (s < 0) continue;
                const double sg = adjb[i * D + q] ? -1.0 : 1.0;
                Fx += sg * f_x[s];
                Fy += sg * f_y[s];
                SF += s_f[s];
            }
            const double svxi = fabs(vx[i]) + dt * SF / m[i], svyi = fabs(vy[i]) + dt * SF / m[i];
            if (svx) svx[i] = svxi;
            if (svy) svy[i] = svyi;
            if (sx) sx[i] = fabs(x[i]) + dt * svxi;
            if (sy) sy[i] = fabs(y[i]) + dt * svyi;
            vx[i] += Fx / m[i] * dt;
            vy[i] += Fy / m[i] * dt;
            x[i] += vx[i] * dt;
            y[i] += vy[i] * dt;
        }
    }
    for (long long s = 0; s < S; s++) {
        if (fx) fx[s] = f_x[s];
        if (fy) fy[s] = f_y[s];
        if (sf) sf[s] = s_f[s];
    }
    free(f_x); free(f_y); free(s_f); free(snap);
    return err ? -err - 10 : nbroken;
}
