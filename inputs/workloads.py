"""Initial states of the workloads, built from the counter-based generator.

Recipes (stated once here and repeated in the design notes):

* Game of Life: W x H torus, cell index y*W + x, a cell starts alive iff its
  uniform draw is below the density (0.25).
* n-body: N bodies, radius sqrt(u1) and angle 2*pi*u2 (uniform in the unit
  disk), mass uniform in [0.5, 1.5], velocity zero.
* spring mesh: W x H jittered grid with spacing h = 1/W centred on the
  origin, jitter uniform in +-0.3 h per coordinate; springs to the right
  neighbour, to the neighbour below and along one random diagonal of every
  grid cell; stiffness 10**U(2, 4); rest length = initial distance; node mass
  1; initial velocity N(0, 0.01**2) per component.
* batched meshes: node counts log-uniform in [1e3, 6.4e4], W = round(sqrt(n)),
  H = ceil(n / W), each mesh built as above with its own seed.
* wa-tor: W x H torus; a cell starts with a fish iff its uniform draw is
  below p_fish, with a shark iff it lies in [p_fish, p_fish + p_shark); the
  agent's spawn timer is uniform in {0 .. its threshold}, a shark's energy is
  energy0.

Everything is produced in float64 and rounded to float32 where the simulated
state is float32; both the oracle and the GPU receive the rounded values.
"""

import math

import numpy as np

from .rng import GAMMA, MASK64, _mix_int, config_seed, normal, uniform

MAX_DEGREE = 8


def gol_init(W: int, H: int, seed: int | None = None, density: float = 0.25) -> np.ndarray:
    """uint8 array of W*H initial cell states (1 = alive), index y*W + x."""
    if seed is None:
        seed = config_seed(1)
    u = uniform(seed, 0, np.arange(W * H))
    return (u < density).astype(np.uint8)


def nbody_init(N: int, seed: int | None = None) -> dict:
    """Positions uniform in the unit disk, masses in [0.5, 1.5], zero velocity (float32)."""
    if seed is None:
        seed = config_seed(2)
    ids = np.arange(N)
    r = np.sqrt(uniform(seed, 0, ids))
    th = 2.0 * np.pi * uniform(seed, 1, ids)
    m = 0.5 + uniform(seed, 2, ids)
    f32 = np.float32
    return {
        "x": (r * np.cos(th)).astype(f32),
        "y": (r * np.sin(th)).astype(f32),
        "vx": np.zeros(N, f32),
        "vy": np.zeros(N, f32),
        "m": m.astype(f32),
    }


def spring_mesh(W: int, H: int, seed: int | None = None, jitter: float = 0.3,
                v_sigma: float = 0.01, id_offset: int = 0, spring_offset: int = 0) -> dict:
    """Jittered planar grid mesh with one random diagonal per cell.

    Returned arrays (float32 state, int32 topology):
      x, y, vx, vy, m          per node (node id = j*W + i + id_offset)
      a, b, k, L0              per spring (spring id = position + spring_offset)
      adj (N, 8), adj_is_b     per node: spring ids in ascending order, -1 = empty
      slot_a, slot_b           per spring: its slot in the adjacency of a / b
    Node and spring ids inside the arrays are local (0-based); the offsets are
    returned for callers that concatenate several meshes.
    """
    if seed is None:
        seed = config_seed(3)
    N = W * H
    ids = np.arange(N, dtype=np.int64)
    i = ids % W
    j = ids // W
    h = 1.0 / W
    jx = (2.0 * uniform(seed, 0, ids) - 1.0) * jitter
    jy = (2.0 * uniform(seed, 1, ids) - 1.0) * jitter
    x = ((i + 0.5 + jx) * h - 0.5 * W * h).astype(np.float32)
    y = ((j + 0.5 + jy) * h - 0.5 * H * h).astype(np.float32)

    has_r = i + 1 < W
    has_d = j + 1 < H
    has_g = has_r & has_d
    coin = uniform(seed, 2, ids) < 0.5
    a = np.stack([ids, ids, np.where(coin, ids, ids + 1)], axis=1)
    b = np.stack([ids + 1, ids + W, np.where(coin, ids + W + 1, ids + W)], axis=1)
    valid = np.stack([has_r, has_d, has_g], axis=1)
    a = a[valid]
    b = b[valid]
    S = a.shape[0]
    sid = np.arange(S, dtype=np.int64)

    k = (10.0 ** (2.0 + 2.0 * uniform(seed, 3, sid))).astype(np.float32)
    dx = x[b].astype(np.float64) - x[a].astype(np.float64)
    dy = y[b].astype(np.float64) - y[a].astype(np.float64)
    L0 = np.sqrt(dx * dx + dy * dy).astype(np.float32)

    node = np.concatenate([a, b])
    spr = np.concatenate([sid, sid])
    isb = np.concatenate([np.zeros(S, np.uint8), np.ones(S, np.uint8)])
    order = np.lexsort((spr, node))
    node_s, spr_s, isb_s = node[order], spr[order], isb[order]
    first = np.searchsorted(node_s, node_s, side="left")
    rank = np.arange(node_s.shape[0]) - first
    if N and rank.max(initial=0) >= MAX_DEGREE:
        raise ValueError("node degree above 8")
    adj = np.full((N, MAX_DEGREE), -1, dtype=np.int32)
    adj_is_b = np.zeros((N, MAX_DEGREE), dtype=np.uint8)
    adj[node_s, rank] = spr_s
    adj_is_b[node_s, rank] = isb_s
    slot_a = np.empty(S, np.int32)
    slot_b = np.empty(S, np.int32)
    sel = isb_s == 0
    slot_a[spr_s[sel]] = rank[sel]
    slot_b[spr_s[~sel]] = rank[~sel]

    vx = (v_sigma * normal(seed, 4, ids)).astype(np.float32)
    vy = (v_sigma * normal(seed, 5, ids)).astype(np.float32)
    return {
        "W": W, "H": H, "N": N, "S": S, "h": h,
        "id_offset": id_offset, "spring_offset": spring_offset,
        "x": x, "y": y, "vx": vx, "vy": vy, "m": np.ones(N, np.float32),
        "a": a.astype(np.int32), "b": b.astype(np.int32), "k": k, "L0": L0,
        "adj": adj, "adj_is_b": adj_is_b, "slot_a": slot_a, "slot_b": slot_b,
    }


def wator_init(W: int, H: int, seed: int | None = None, p_fish: float = 0.3, p_shark: float = 0.05,
               fish_spawn: int = 4, shark_spawn: int = 12, energy0: int = 8) -> dict:
    """Initial wa-tor agents per cell index y*W + x: kind (u8: 0 empty, 1 fish,
    2 shark), timer and energy (i32; 0 where they do not apply)."""
    if seed is None:
        seed = config_seed(6)
    ids = np.arange(W * H)
    u = uniform(seed, 0, ids)
    kind = np.where(u < p_fish, 1, np.where(u < p_fish + p_shark, 2, 0)).astype(np.uint8)
    v = uniform(seed, 1, ids)
    thr = np.where(kind == 1, fish_spawn, shark_spawn)
    timer = np.where(kind > 0, np.floor(v * (thr + 1)), 0).astype(np.int32)
    energy = np.where(kind == 2, energy0, 0).astype(np.int32)
    return {"kind": kind, "timer": timer, "energy": energy}


def struct_seed(base: int, s: int) -> int:
    return _mix_int((base + GAMMA * (s + 1)) & MASK64)


def batched_sizes(n_struct: int = 256, seed: int | None = None,
                  lo: float = 1e3, hi: float = 6.4e4) -> list:
    """(W, H) of each structure: n log-uniform in [lo, hi], W = round(sqrt(n)), H = ceil(n/W)."""
    if seed is None:
        seed = config_seed(4)
    u = uniform(seed, 0, np.arange(n_struct))
    n = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    out = []
    for nn in n:
        W = int(round(math.sqrt(int(nn))))
        H = int(math.ceil(int(nn) / W))
        out.append((W, H))
    return out


def batched_meshes(n_struct: int = 256, seed: int | None = None,
                   lo: float = 1e3, hi: float = 6.4e4) -> list:
    """List of independent meshes with global id offsets (nodes and springs)."""
    if seed is None:
        seed = config_seed(4)
    meshes = []
    noff = 0
    soff = 0
    for s, (W, H) in enumerate(batched_sizes(n_struct, seed, lo, hi)):
        m = spring_mesh(W, H, struct_seed(seed, s), id_offset=noff, spring_offset=soff)
        meshes.append(m)
        noff += m["N"]
        soff += m["S"]
    return meshes


def concat_meshes(meshes: list) -> dict:
    """One mesh dict holding independent meshes side by side: node and spring
    ids are shifted by the sizes of the meshes before (global ids); slots are
    unchanged.  Springs of one mesh only reference that mesh's nodes."""
    out = {}
    for key in ("x", "y", "vx", "vy", "m", "k", "L0", "slot_a", "slot_b"):
        out[key] = np.concatenate([m[key] for m in meshes])
    noff = np.cumsum([0] + [m["N"] for m in meshes])
    soff = np.cumsum([0] + [m["S"] for m in meshes])
    out["a"] = np.concatenate([m["a"] + noff[i] for i, m in enumerate(meshes)]).astype(np.int32)
    out["b"] = np.concatenate([m["b"] + noff[i] for i, m in enumerate(meshes)]).astype(np.int32)
    out["adj"] = np.concatenate([np.where(m["adj"] >= 0, m["adj"] + soff[i], -1)
                                 for i, m in enumerate(meshes)]).astype(np.int32)
    out["adj_is_b"] = np.concatenate([m["adj_is_b"] for m in meshes])
    out["N"] = int(noff[-1])
    out["S"] = int(soff[-1])
    out["node_offsets"] = noff
    out["spring_offsets"] = soff
    return out


def structure_mesh(W: int, H: int, seed: int | None = None, jitter: float = 0.2, pull_speed: float = 0.5,
                   break_strain: float = 0.04, break_spread: float = 0.5, v_sigma: float = 0.0,
                   stretch_rate: float = 0.0) -> dict:
    """Mesh of the fracture simulation ("structure"): a W x H brick-wall
    lattice (every node has springs to its left and right neighbours and, on
    alternating columns, to the node above or below: at most three springs per
    node), jittered positions with spacing h = 1/W.  Column 0 holds anchor
    nodes, column W-1 pull nodes moving at (pull_speed, 0), the rest ordinary
    nodes of mass 1 at rest (or with N(0, v_sigma^2) velocities), plus
    vx = stretch_rate * x (a uniform stretch of the whole mesh).  Spring
    stiffness k = 10^U(2, 3); rest length L0 = initial length; force limit
    k * L0 * break_strain * (1 + break_spread * U(-1, 1)).

    Returned arrays (float32 state, int32 topology; node id = j*W + i):
      ntype (0 anchor, 1 pull, 2 node), nalive, x, y, vx, vy, m,
      slot (N*3 spring ids, -1 empty), isp2 (N*3), nspr, dist,
      p1, p2, k, L0, maxf, s1, s2, salive (spring id = position).
    """
    if seed is None:
        seed = config_seed(6)
    N = W * H
    ids = np.arange(N, dtype=np.int64)
    i = ids % W
    j = ids // W
    h = 1.0 / W
    x = ((i + (2.0 * uniform(seed, 0, ids) - 1.0) * jitter) * h).astype(np.float32)
    y = ((j + (2.0 * uniform(seed, 1, ids) - 1.0) * jitter) * h).astype(np.float32)
    ntype = np.full(N, 2, np.int32)
    ntype[i == W - 1] = 1
    ntype[i == 0] = 0
    vx = np.zeros(N, np.float32)
    vy = np.zeros(N, np.float32)
    if v_sigma > 0:
        vx = (v_sigma * normal(seed, 2, ids)).astype(np.float32)
        vy = (v_sigma * normal(seed, 3, ids)).astype(np.float32)
        vx[ntype == 0] = 0
        vy[ntype == 0] = 0
    if stretch_rate:
        vx = (vx + stretch_rate * x).astype(np.float32)
        vx[ntype == 0] = 0
    vx[ntype == 1] = pull_speed
    vy[ntype == 1] = 0
    # horizontal springs, then the vertical ones of the columns with (i + j) even
    hor = ids[i + 1 < W]
    ver = ids[((i + j) % 2 == 0) & (j + 1 < H)]
    p1 = np.concatenate([hor, ver])
    p2 = np.concatenate([hor + 1, ver + W])
    S = p1.size
    sid = np.arange(S, dtype=np.int64)
    k = (10.0 ** (2.0 + uniform(seed, 4, sid))).astype(np.float32)
    dx = x[p2].astype(np.float64) - x[p1].astype(np.float64)
    dy = y[p2].astype(np.float64) - y[p1].astype(np.float64)
    L0 = np.sqrt(dx * dx + dy * dy).astype(np.float32)
    maxf = (k.astype(np.float64) * L0 * break_strain
            * (1.0 + break_spread * (2.0 * uniform(seed, 5, sid) - 1.0))).astype(np.float32)
    node = np.concatenate([p1, p2])
    spr = np.concatenate([sid, sid])
    isb = np.concatenate([np.zeros(S, np.uint8), np.ones(S, np.uint8)])
    order = np.lexsort((spr, node))
    node_s, spr_s, isb_s = node[order], spr[order], isb[order]
    first = np.searchsorted(node_s, node_s, side="left")
    rank = np.arange(node_s.size) - first
    if N and rank.max(initial=0) >= 3:
        raise ValueError("node degree above 3")
    slot = np.full((N, 3), -1, np.int32)
    isp2 = np.zeros((N, 3), np.uint8)
    slot[node_s, rank] = spr_s
    isp2[node_s, rank] = isb_s
    s1 = np.empty(S, np.int32)
    s2 = np.empty(S, np.int32)
    sel = isb_s == 0
    s1[spr_s[sel]] = rank[sel]
    s2[spr_s[~sel]] = rank[~sel]
    return {
        "ntype": ntype, "nalive": np.ones(N, np.uint8), "x": x, "y": y, "vx": vx, "vy": vy,
        "m": np.ones(N, np.float32), "slot": slot.reshape(-1), "isp2": isp2.reshape(-1),
        "nspr": (slot >= 0).sum(axis=1).astype(np.int32), "dist": np.zeros(N, np.int32),
        "p1": p1.astype(np.int32), "p2": p2.astype(np.int32), "k": k, "L0": L0, "maxf": maxf,
        "s1": s1, "s2": s2, "salive": np.ones(S, np.uint8),
    }


def hub_mesh(W: int, H: int, hubs: int = 8, hub_springs: int = 32, seed: int | None = None, **kw) -> dict:
    """spring_mesh(W, H) plus `hub_springs` extra springs from each of `hubs`
    hub nodes to other nodes drawn at random (stiffness 10^U(2,4), rest length
    the initial distance): a mesh of high-degree nodes.  adj / adj_is_b have
    shape (N, D) with D the largest degree; slots in spring-id order; the
    extra springs follow the mesh's springs in id order."""
    if seed is None:
        seed = config_seed(7)
    m = spring_mesh(W, H, seed=seed, **kw)
    N = W * H
    hub_ids = np.unique((uniform(seed, 10, np.arange(hubs)) * N).astype(np.int64) % max(N, 1))
    src, dst = [], []
    for h in hub_ids:
        j = np.arange(hub_springs, dtype=np.int64)
        t = (uniform(seed, 11 + int(h) % 1000, j + int(h) * hub_springs) * N).astype(np.int64) % N
        t = np.unique(t[t != h])
        src.append(np.full(t.size, h))
        dst.append(t)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    dst = np.concatenate(dst) if dst else np.zeros(0, np.int64)
    a0 = np.asarray(m["a"], np.int64)
    b0 = np.asarray(m["b"], np.int64)
    # no duplicate of an existing spring
    key0 = set(zip(np.minimum(a0, b0).tolist(), np.maximum(a0, b0).tolist()))
    keep = np.array([(min(s, d), max(s, d)) not in key0 for s, d in zip(src.tolist(), dst.tolist())], bool)
    if keep.size:
        src, dst = src[keep], dst[keep]
    a = np.concatenate([a0, np.minimum(src, dst)])
    b = np.concatenate([b0, np.maximum(src, dst)])
    S = a.size
    sid = np.arange(S, dtype=np.int64)
    x = np.asarray(m["x"])
    y = np.asarray(m["y"])
    kx = (10.0 ** (2.0 + 2.0 * uniform(seed, 12, sid[a0.size:]))).astype(np.float32)
    k = np.concatenate([np.asarray(m["k"], np.float32), kx])
    dx = x[b].astype(np.float64) - x[a].astype(np.float64)
    dy = y[b].astype(np.float64) - y[a].astype(np.float64)
    L0 = np.sqrt(dx * dx + dy * dy).astype(np.float32)
    node = np.concatenate([a, b])
    spr = np.concatenate([sid, sid])
    isb = np.concatenate([np.zeros(S, np.uint8), np.ones(S, np.uint8)])
    order = np.lexsort((spr, node))
    node_s, spr_s, isb_s = node[order], spr[order], isb[order]
    first = np.searchsorted(node_s, node_s, side="left")
    rank = np.arange(node_s.size) - first
    D = int(rank.max(initial=0)) + 1
    adj = np.full((N, D), -1, np.int32)
    adj_is_b = np.zeros((N, D), np.uint8)
    adj[node_s, rank] = spr_s
    adj_is_b[node_s, rank] = isb_s
    slot_a = np.empty(S, np.int32)
    slot_b = np.empty(S, np.int32)
    sel = isb_s == 0
    slot_a[spr_s[sel]] = rank[sel]
    slot_b[spr_s[~sel]] = rank[~sel]
    out = dict(m)
    out.update(a=a.astype(np.int32), b=b.astype(np.int32), k=k, L0=L0, adj=adj, adj_is_b=adj_is_b,
               slot_a=slot_a, slot_b=slot_b, S=int(S))
    return out
