"""ctypes wrapper of the C oracle (smmo_oracle.c).  TEST INFRASTRUCTURE ONLY.

Each function names the thesis passage that its C counterpart follows; the
C file carries the full statement of the semantics.
"""

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smmo_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build() -> str:
    """Compile the oracle with gcc (always recompiles).  Returns the library path."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = C.CDLL(_LIB)
            P = C.c_void_p
            LL = C.c_longlong
            D = C.c_double
            lib.orc_gol_create.restype = P
            lib.orc_gol_create.argtypes = [C.c_int, C.c_int, P]
            lib.orc_gol_step.restype = C.c_int
            lib.orc_gol_step.argtypes = [P, C.c_int]
            lib.orc_gol_read.restype = LL
            lib.orc_gol_read.argtypes = [P, P, P, P]
            lib.orc_gol_error.restype = C.c_int
            lib.orc_gol_error.argtypes = [P]
            lib.orc_gol_free.restype = None
            lib.orc_gol_free.argtypes = [P]
            lib.orc_nbody_steps.restype = C.c_int
            lib.orc_nbody_steps.argtypes = [LL, P, P, P, P, P, P, P, D, D, D, C.c_int, P, P]
            lib.orc_nbody_update.restype = C.c_int
            lib.orc_nbody_update.argtypes = [LL, P, P, P, P, P, P, P, D]
            lib.orc_nbody_force_at.restype = C.c_int
            lib.orc_nbody_force_at.argtypes = [LL, P, P, P, D, D, P, LL, P, P, P, P]
            lib.orc_spring_steps.restype = LL
            lib.orc_spring_steps.argtypes = [LL, P, P, P, P, P, P, P, LL, P, P, P, P, P, P,
                                             P, P, P, D, D, C.c_int, P, P, P, P, P, C.c_int, P, P]
            lib.orc_spring_adjoint.restype = C.c_int
            lib.orc_spring_adjoint.argtypes = [LL, P, P, P, P, P, P, P, LL, P, P, P, P, P, P, P, P,
                                               D, C.c_int, C.c_int, P, P, P, P, P, P, P, P, P]
            lib.orc_spring_adjoint_step.restype = C.c_int
            lib.orc_spring_adjoint_step.argtypes = [LL, P, P, P, P, P, LL, P, P, P, P, D,
                                                    P, P, P, P, P, P, P, P, P, P]
            lib.orc_spring_breaks.restype = C.c_int
            lib.orc_spring_breaks.argtypes = [D, D, D, D, D, D, P]
            lib.orc_spring_tie_band.restype = D
            lib.orc_spring_tie_band.argtypes = []
            lib.orc_threads.restype = C.c_int
            lib.orc_threads.argtypes = []
            lib.orc_set_threads.restype = None
            lib.orc_set_threads.argtypes = [C.c_int]
            lib.orc_wator_create.restype = P
            lib.orc_wator_create.argtypes = [C.c_int, C.c_int, C.c_uint64, P, P, P, P]
            lib.orc_wator_step.restype = C.c_int
            lib.orc_wator_step.argtypes = [P, C.c_int]
            lib.orc_wator_read.restype = C.c_int
            lib.orc_wator_read.argtypes = [P, P, P, P, P]
            lib.orc_wator_free.restype = None
            lib.orc_wator_free.argtypes = [P]
            lib.orc_spring_steps_deg.restype = LL
            lib.orc_spring_steps_deg.argtypes = [LL, C.c_int, P, P, P, P, P, P, P, LL, P, P, P, P, P, P,
                                                 P, P, P, D, D, C.c_int, P, P, P, P, P, P, P]
            lib.orc_generation_steps.restype = C.c_int
            lib.orc_generation_steps.argtypes = [C.c_int, C.c_int, P, P, C.c_uint32, C.c_uint32, C.c_int32,
                                                 C.c_int]
            lib.orc_structure_pull.restype = C.c_int
            lib.orc_structure_pull.argtypes = [LL, P, P, P, P, P, P, D]
            lib.orc_structure_step.restype = LL
            lib.orc_structure_step.argtypes = [LL, P, P, P, P, P, P, P, P, P, P, LL, P, P, P, P, P, P, P,
                                               P, P, P, D, P, P, P, P, P, P, P]
            lib.orc_structure_bfs.restype = LL
            lib.orc_structure_bfs.argtypes = [LL, P, P, P, P, P, P, LL, P, P, P, P, P, P, P]
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).copy()


class GolWorld:
    """Game of Life in SMMO form on a W x H torus (thesis Ch.7 "gol", rule B3/S23)."""

    def __init__(self, W: int, H: int, init):
        self.lib = _load()
        self.W, self.H = W, H
        init = np.ascontiguousarray(init, dtype=np.uint8).reshape(-1)
        assert init.size == W * H
        self._init = init
        self.h = self.lib.orc_gol_create(W, H, _p(init))
        if not self.h:
            raise ValueError("bad grid")

    def step(self, n: int = 1):
        err = self.lib.orc_gol_step(self.h, n)
        if err:
            raise RuntimeError("oracle gol error %d" % err)

    def read(self):
        """(state u8[W*H], count i32[W*H], sorted cell indices of Alive objects)."""
        nc = self.W * self.H
        st = np.empty(nc, np.uint8)
        ct = np.empty(nc, np.int32)
        al = np.empty(nc, np.int32)
        n = self.lib.orc_gol_read(self.h, _p(st), _p(ct), _p(al))
        if self.lib.orc_gol_error(self.h):
            raise RuntimeError("oracle gol error %d" % self.lib.orc_gol_error(self.h))
        return st, ct, al[:n].copy()

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_gol_free(self.h)
            self.h = None


class WatorWorld:
    """wa-tor in SMMO form on a W x H torus (thesis Ch.7 "wa-tor"): Cell, Fish
    and Shark objects, eight do-alls per iteration.  params = (fish_spawn,
    shark_spawn, energy0, boost); init = dict of per-cell arrays kind (0
    empty, 1 fish, 2 shark), timer and energy; seed keys the random choices."""

    def __init__(self, W: int, H: int, seed: int, params, init: dict):
        self.lib = _load()
        self.W, self.H = W, H
        nc = W * H
        self._keep = [np.ascontiguousarray(init["kind"], dtype=np.uint8),
                      np.ascontiguousarray(init["timer"], dtype=np.int32),
                      np.ascontiguousarray(init["energy"], dtype=np.int32),
                      np.ascontiguousarray(params, dtype=np.int32)]
        assert all(a.size == nc for a in self._keep[:3]) and self._keep[3].size == 4
        kind, timer, energy, prm = self._keep
        self.h = self.lib.orc_wator_create(W, H, seed, _p(prm), _p(kind), _p(timer), _p(energy))
        if not self.h:
            raise ValueError("bad grid")

    def step(self, n: int = 1):
        err = self.lib.orc_wator_step(self.h, n)
        if err:
            raise RuntimeError("oracle wa-tor error %d" % err)

    def read(self):
        """Per cell index: kind (u8), spawn timer and energy (i32, 0 where no
        agent / no shark); plus (live fish, live sharks)."""
        nc = self.W * self.H
        kind = np.empty(nc, np.uint8)
        timer = np.empty(nc, np.int32)
        energy = np.empty(nc, np.int32)
        counts = np.empty(2, np.int64)
        err = self.lib.orc_wator_read(self.h, _p(kind), _p(timer), _p(energy), _p(counts))
        if err:
            raise RuntimeError("oracle wa-tor error %d" % err)
        return kind, timer, energy, (int(counts[0]), int(counts[1]))

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_wator_free(self.h)
            self.h = None


def nbody_steps(x, y, vx, vy, m, G, eps, dt, steps=1):
    """Thesis Ch.7 "nbody": `steps` x {compute_force (device_do), update}, float64.

    Returns dict of x, y, vx, vy, fx, fy and the force conditioning scales
    sfx, sfy = sum_j |term_ij| of the last force evaluation.
    """
    lib = _load()
    x, y, vx, vy, m = (_f64(a) for a in (x, y, vx, vy, m))
    n = x.size
    fx, fy, sfx, sfy = (np.zeros(n) for _ in range(4))
    rc = lib.orc_nbody_steps(n, _p(x), _p(y), _p(vx), _p(vy), _p(fx), _p(fy), _p(m),
                             float(G), float(eps), float(dt), int(steps), _p(sfx), _p(sfy))
    if rc:
        raise RuntimeError("oracle nbody error %d" % rc)
    return dict(x=x, y=y, vx=vx, vy=vy, fx=fx, fy=fy, sfx=sfx, sfy=sfy)


def nbody_update(x, y, vx, vy, fx, fy, m, dt):
    """Body::update alone from given forces: v += f/m dt, x += v dt (float64)."""
    lib = _load()
    x, y, vx, vy, fx, fy, m = (_f64(a) for a in (x, y, vx, vy, fx, fy, m))
    rc = lib.orc_nbody_update(x.size, _p(x), _p(y), _p(vx), _p(vy), _p(fx), _p(fy), _p(m), float(dt))
    if rc:
        raise RuntimeError("oracle nbody error %d" % rc)
    return dict(x=x, y=y, vx=vx, vy=vy)


def nbody_force_at(x, y, m, G, eps, idx):
    """compute_force of the bodies `idx` only: (fx, fy, sfx, sfy), float64."""
    lib = _load()
    x, y, m = (_f64(a) for a in (x, y, m))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    k = idx.size
    fx, fy, sfx, sfy = (np.zeros(k) for _ in range(4))
    rc = lib.orc_nbody_force_at(x.size, _p(x), _p(y), _p(m), float(G), float(eps),
                                _p(idx), k, _p(fx), _p(fy), _p(sfx), _p(sfy))
    if rc:
        raise RuntimeError("oracle nbody error %d" % rc)
    return fx, fy, sfx, sfy


def _ties(tie, S):
    if tie is None:
        return None
    t = np.ascontiguousarray(tie, dtype=np.int8)
    assert t.size == S
    return t


def set_threads(n: int) -> None:
    """Host threads for the oracle's parallel do-alls from now on."""
    _load().orc_set_threads(int(n))


def threads() -> int:
    """Host threads the oracle's parallel do-alls use (OMP_NUM_THREADS)."""
    return int(_load().orc_threads())


def spring_tie_band() -> float:
    """Half-width of the band of strains around the break threshold within
    which either break decision is correct (float32 rounding of the strain)."""
    return float(_load().orc_spring_tie_band())


def spring_steps(mesh: dict, dt: float, thresh: float = 0.3, steps: int = 1,
                 alive=None, fx=None, fy=None, tension_only: bool = False, tie=None):
    """Thesis Ch.7 "structure" compute steps: `steps` x {Spring::compute_force,
    Node::update} in float64, the break rule (strain > thresh) decided in
    float64; tension_only = springs that only pull (no force while l <= L0).

    `mesh` holds x, y, vx, vy, m, adj, adj_is_b, a, b, k, L0, slot_a, slot_b
    (ids local to the arrays).  tie (int8 per spring, optional): fixed break
    decisions (0 keep, 1 break, -1 decide) of springs within the tie band in
    the first step.  Returns a new dict with the updated state, the spring
    forces fx, fy, the alive flags, the number of springs broken, the strain
    of each spring at its last force pass (NaN for springs dead at the start)
    and the conditioning scales sf (per spring), svx, svy, sx, sy (per node).
    """
    lib = _load()
    N = int(np.asarray(mesh["x"]).size)
    S = int(np.asarray(mesh["a"]).size)
    x, y, vx, vy, m = (_f64(mesh[k]) for k in ("x", "y", "vx", "vy", "m"))
    adj = np.ascontiguousarray(mesh["adj"], dtype=np.int32).reshape(N, 8).copy()
    adjb = np.ascontiguousarray(mesh["adj_is_b"], dtype=np.uint8).reshape(N, 8)
    a = np.ascontiguousarray(mesh["a"], dtype=np.int32)
    b = np.ascontiguousarray(mesh["b"], dtype=np.int32)
    kk = _f64(mesh["k"])
    L0 = _f64(mesh["L0"])
    sa = np.ascontiguousarray(mesh["slot_a"], dtype=np.int32)
    sb = np.ascontiguousarray(mesh["slot_b"], dtype=np.int32)
    al = (np.ones(S, np.uint8) if alive is None else np.ascontiguousarray(alive, dtype=np.uint8).copy())
    fxo = np.zeros(S) if fx is None else _f64(fx)
    fyo = np.zeros(S) if fy is None else _f64(fy)
    sf = np.zeros(S)
    strain = np.full(S, np.nan)
    svx, svy, sx, sy = (np.zeros(N) for _ in range(4))
    t = _ties(tie, S)
    nb = lib.orc_spring_steps(N, _p(x), _p(y), _p(vx), _p(vy), _p(m), _p(adj), _p(adjb),
                              S, _p(a), _p(b), _p(kk), _p(L0), _p(sa), _p(sb), _p(al),
                              _p(fxo), _p(fyo), float(dt), float(thresh), int(steps),
                              _p(sf), _p(svx), _p(svy), _p(sx), _p(sy), int(bool(tension_only)),
                              _p(t), _p(strain))
    if nb < 0:
        raise RuntimeError("oracle spring error %d" % nb)
    out = dict(mesh)
    out.update(x=x, y=y, vx=vx, vy=vy, adj=adj, alive=al, fx=fxo, fy=fyo, nbroken=int(nb),
               sf=sf, svx=svx, svy=svy, sx=sx, sy=sy, strain=strain)
    return out


def spring_steps_deg(mesh: dict, dt: float, thresh: float = 0.3, steps: int = 1, alive=None, fx=None, fy=None,
                     tie=None):
    """spring_steps for meshes of any node degree D (adj and adj_is_b of shape
    (N, D)): the same steps and decisions, slots summed in order."""
    lib = _load()
    adj = np.array(mesh["adj"], dtype=np.int32, copy=True)
    N = int(np.asarray(mesh["x"]).size)
    adj = adj.reshape(N, -1)
    D = adj.shape[1]
    S = int(np.asarray(mesh["a"]).size)
    x, y, vx, vy, m = (_f64(mesh[k]) for k in ("x", "y", "vx", "vy", "m"))
    adjb = np.ascontiguousarray(mesh["adj_is_b"], dtype=np.uint8).reshape(N, D)
    a = np.ascontiguousarray(mesh["a"], dtype=np.int32)
    b = np.ascontiguousarray(mesh["b"], dtype=np.int32)
    kk = _f64(mesh["k"])
    L0 = _f64(mesh["L0"])
    sa = np.ascontiguousarray(mesh["slot_a"], dtype=np.int32)
    sb = np.ascontiguousarray(mesh["slot_b"], dtype=np.int32)
    al = (np.ones(S, np.uint8) if alive is None else np.ascontiguousarray(alive, dtype=np.uint8).copy())
    fxo = np.zeros(S) if fx is None else _f64(fx)
    fyo = np.zeros(S) if fy is None else _f64(fy)
    sf = np.zeros(S)
    strain = np.full(S, np.nan)
    svx, svy, sx, sy = (np.zeros(N) for _ in range(4))
    t = _ties(tie, S)
    nb = lib.orc_spring_steps_deg(N, D, _p(x), _p(y), _p(vx), _p(vy), _p(m), _p(adj), _p(adjb), S, _p(a), _p(b),
                                  _p(kk), _p(L0), _p(sa), _p(sb), _p(al), _p(fxo), _p(fyo), float(dt),
                                  float(thresh), int(steps), _p(sf), _p(svx), _p(svy), _p(sx), _p(sy),
                                  _p(t), _p(strain))
    if nb < 0:
        raise RuntimeError("oracle spring error %d" % nb)
    out = dict(mesh)
    out.update(x=x, y=y, vx=vx, vy=vy, adj=adj, alive=al, fx=fxo, fy=fyo, nbroken=int(nb),
               sf=sf, svx=svx, svy=svy, sx=sx, sy=sy, strain=strain)
    return out


def spring_breaks(xa, ya, xb, yb, L0, thresh=0.3, with_strain=False):
    """The break decision of one spring (float64: strain (l - L0)/L0 > thresh);
    with_strain: (decision, strain)."""
    e = C.c_double()
    r = bool(_load().orc_spring_breaks(float(xa), float(ya), float(xb), float(yb),
                                       float(L0), float(thresh), C.byref(e)))
    return (r, e.value) if with_strain else r


def spring_adjoint(mesh: dict, dt: float, steps: int, every: int = 20, xhat=None, yhat=None):
    """Reverse-mode gradients of L = 1/2 |x_T - xhat|^2 through `steps`
    spring-mesh steps with breaking off (float64), checkpointing (x, v) every
    `every` steps.  xhat defaults to the initial positions.  Returns dict with
    loss, gk (dL/dk), gvx, gvy (dL/dv0), gx, gy (dL/dx0), xT, yT, and agk =
    sum over the reverse steps of dt |g| per spring, g = w_a - w_b (it bounds
    the factor dt |u . g| of each step's stretch in dL/dk: an error e in every
    stretch l - L0 moves dL/dk by at most e agk)."""
    lib = _load()
    N = int(np.asarray(mesh["x"]).size)
    S = int(np.asarray(mesh["a"]).size)
    x, y, vx, vy, m = (_f64(mesh[k]) for k in ("x", "y", "vx", "vy", "m"))
    adj = np.ascontiguousarray(mesh["adj"], dtype=np.int32).reshape(N, 8)
    adjb = np.ascontiguousarray(mesh["adj_is_b"], dtype=np.uint8).reshape(N, 8)
    a = np.ascontiguousarray(mesh["a"], dtype=np.int32)
    b = np.ascontiguousarray(mesh["b"], dtype=np.int32)
    kk = _f64(mesh["k"])
    L0 = _f64(mesh["L0"])
    sa = np.ascontiguousarray(mesh["slot_a"], dtype=np.int32)
    sb = np.ascontiguousarray(mesh["slot_b"], dtype=np.int32)
    xh = x.copy() if xhat is None else _f64(xhat)
    yh = y.copy() if yhat is None else _f64(yhat)
    gk, agk = np.zeros(S), np.zeros(S)
    gvx, gvy, gx, gy, xT, yT = (np.zeros(N) for _ in range(6))
    loss = C.c_double()
    rc = lib.orc_spring_adjoint(N, _p(x), _p(y), _p(vx), _p(vy), _p(m), _p(adj), _p(adjb), S, _p(a),
                                _p(b), _p(kk), _p(L0), _p(sa), _p(sb), _p(xh), _p(yh), float(dt),
                                int(steps), int(every), _p(gk), _p(gvx), _p(gvy), _p(gx), _p(gy),
                                _p(xT), _p(yT), C.byref(loss), _p(agk))
    if rc:
        raise RuntimeError("oracle adjoint error %d" % rc)
    return dict(loss=loss.value, gk=gk, gvx=gvx, gvy=gvy, gx=gx, gy=gy, xT=xT, yT=yT, agk=agk)


def spring_adjoint_step(mesh: dict, px, py, dt, lx, ly, lvx, lvy):
    """One reverse step from positions x_n (px, py) and the adjoints at step
    n+1; returns the adjoints at step n, this step's dL/dk contribution and
    the conditioning scales (sgk, slx, sly, slvx, slvy)."""
    lib = _load()
    N = int(np.asarray(mesh["x"]).size)
    S = int(np.asarray(mesh["a"]).size)
    px, py, m = _f64(px), _f64(py), _f64(mesh["m"])
    adj = np.ascontiguousarray(mesh["adj"], dtype=np.int32).reshape(N, 8)
    adjb = np.ascontiguousarray(mesh["adj_is_b"], dtype=np.uint8).reshape(N, 8)
    a = np.ascontiguousarray(mesh["a"], dtype=np.int32)
    b = np.ascontiguousarray(mesh["b"], dtype=np.int32)
    kk, L0 = _f64(mesh["k"]), _f64(mesh["L0"])
    lx, ly, lvx, lvy = (_f64(v) for v in (lx, ly, lvx, lvy))
    gk, sgk = np.zeros(S), np.zeros(S)
    slx, sly, slvx, slvy = (np.zeros(N) for _ in range(4))
    rc = lib.orc_spring_adjoint_step(N, _p(px), _p(py), _p(m), _p(adj), _p(adjb), S, _p(a), _p(b),
                                     _p(kk), _p(L0), float(dt), _p(lx), _p(ly), _p(lvx), _p(lvy),
                                     _p(gk), _p(sgk), _p(slx), _p(sly), _p(slvx), _p(slvy))
    if rc:
        raise RuntimeError("oracle adjoint step error %d" % rc)
    return dict(lx=lx, ly=ly, lvx=lvx, lvy=lvy, gk=gk, sgk=sgk, slx=slx, sly=sly, slvx=slvx, slvy=slvy)


# ---------------------------------------------------------------- structure --
STRUCTURE_ANCHOR, STRUCTURE_PULL, STRUCTURE_NODE = 0, 1, 2
STRUCTURE_MAXDIST = 0x7FFFFFFF


def _structure_arrays(st: dict) -> dict:
    """Private, contiguous copies of a structure state (see structure_step)."""
    N = int(np.asarray(st["x"]).size)
    S = int(np.asarray(st["p1"]).size)
    c = lambda a, dt: np.array(a, dtype=dt, copy=True).reshape(-1)
    out = dict(st)
    for key in ("x", "y", "vx", "vy", "m"):
        out[key] = c(st[key], np.float64)
    for key in ("k", "L0", "maxf"):
        out[key] = c(st[key], np.float64)
    out["fx"] = c(st.get("fx", np.zeros(S)), np.float64)
    out["fy"] = c(st.get("fy", np.zeros(S)), np.float64)
    for key in ("ntype", "nspr", "p1", "p2", "s1", "s2"):
        out[key] = c(st[key], np.int32)
    out["dist"] = c(st.get("dist", np.zeros(N)), np.int32)
    out["slot"] = c(st["slot"], np.int32)
    for key in ("nalive", "salive", "isp2"):
        out[key] = c(st[key], np.uint8)
    out["sdel"] = c(st.get("sdel", np.zeros(S)), np.uint8)
    assert out["slot"].size == 3 * N and out["isp2"].size == 3 * N
    return out


def structure_pull(st: dict, dt: float) -> dict:
    """AnchorPullNode::pull (thesis Ch.7 "structure", step 1) in float64."""
    o = _structure_arrays(st)
    _load().orc_structure_pull(o["x"].size, _p(o["ntype"]), _p(o["nalive"]), _p(o["x"]), _p(o["y"]),
                               _p(o["vx"]), _p(o["vy"]), float(dt))
    return o


STRUCTURE_TIE_REL = 1e-6   # tie band of the force limit, relative to k (l + L0)


def structure_step(st: dict, dt: float, tie=None) -> dict:
    """One compute step of "structure" (Spring::force, then Node::update).

    State: per node id ntype (0 anchor, 1 pull, 2 node), nalive, x, y, vx, vy,
    m, slot (3 per node: spring id or -1), isp2 (3 per node), nspr, dist; per
    spring id p1, p2, k, L0, maxf, s1, s2, salive, fx, fy, sdel.  tie (int8 per
    spring, optional): fixed break decisions of ties.  Returns the new state
    with nbroken, the float64 force F = k (l - L0) of each spring live at the
    start (NaN otherwise) and the conditioning scales sf, svx, svy, sx, sy.
    """
    o = _structure_arrays(st)
    N, S = o["x"].size, o["p1"].size
    sf = np.zeros(S)
    F = np.full(S, np.nan)
    svx, svy, sx, sy = (np.zeros(N) for _ in range(4))
    t = _ties(tie, S)
    nb = _load().orc_structure_step(
        N, _p(o["ntype"]), _p(o["nalive"]), _p(o["x"]), _p(o["y"]), _p(o["vx"]), _p(o["vy"]), _p(o["m"]),
        _p(o["slot"]), _p(o["isp2"]), _p(o["nspr"]), S, _p(o["p1"]), _p(o["p2"]), _p(o["k"]), _p(o["L0"]),
        _p(o["maxf"]), _p(o["s1"]), _p(o["s2"]), _p(o["salive"]), _p(o["fx"]), _p(o["fy"]), float(dt),
        _p(sf), _p(svx), _p(svy), _p(sx), _p(sy), _p(t), _p(F))
    if nb < 0:
        raise RuntimeError("oracle structure error %d" % nb)
    o.update(nbroken=int(nb), sf=sf, svx=svx, svy=svy, sx=sx, sy=sy, F=F)
    return o


def structure_bfs(st: dict) -> dict:
    """Removal of disconnected nodes (thesis Ch.7 "structure", step 3).
    Returns the new state with dist, levels (visit passes) and ndeleted."""
    o = _structure_arrays(st)
    N, S = o["x"].size, o["p1"].size
    lv = C.c_int(0)
    nd = _load().orc_structure_bfs(N, _p(o["ntype"]), _p(o["nalive"]), _p(o["slot"]), _p(o["isp2"]),
                                   _p(o["nspr"]), _p(o["dist"]), S, _p(o["p1"]), _p(o["p2"]), _p(o["s1"]),
                                   _p(o["s2"]), _p(o["salive"]), _p(o["sdel"]), C.byref(lv))
    if nd < 0:
        raise RuntimeError("oracle structure error %d" % nd)
    o.update(levels=int(lv.value), ndeleted=int(nd))
    return o


# --------------------------------------------------------------- generation --
BURST_SURVIVE = (0, 2, 3, 5, 6, 7, 8)
BURST_BIRTH = (3, 4, 6, 8)
BURST_DYING = 255


def _mask(counts) -> int:
    m = 0
    for c in counts:
        m |= 1 << int(c)
    return m


def generation_steps(W: int, H: int, state, left, steps: int = 1, survive=BURST_SURVIVE, birth=BURST_BIRTH,
                     dying: int = BURST_DYING):
    """The generational cellular automaton of thesis Ch.7 "generation" (rule
    Burst by default) on a W x H torus: returns new (state, left) arrays
    (state 0 empty, 1 live, 2 dying; left = dying generations left)."""
    st = np.array(state, dtype=np.uint8, copy=True).reshape(-1)
    lf = np.array(left, dtype=np.int32, copy=True).reshape(-1)
    assert st.size == W * H and lf.size == W * H
    rc = _load().orc_generation_steps(int(W), int(H), _p(st), _p(lf), _mask(survive), _mask(birth), int(dying),
                                      int(steps))
    if rc:
        raise RuntimeError("oracle generation error %d" % rc)
    return st, lf
