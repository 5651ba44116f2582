"""CPU oracle of the time-averaged flux reconstruction step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2512_08611_amd``; the two meet only through the
seeded input generators of ``paper_2512_08611_amd.workloads``, which hold none
of the method's arithmetic.

The numerics live in plain C++ (``oracle/*.hpp``, compiled into
``oracle/liboracle.so`` by ``__graft_entry__.build()``); this module is the
ctypes marshalling plus the Fourier (von Neumann) analysis in ``cfl.py``.

Parity status of each part (what pins it) is listed in the design notes.  The
smoothness indicator constants come from the cited work of Hennemann et al.,
not from the paper; the indicator is pinned by its special cases (constant
state -> 0, pure highest mode -> alpha_max) and by closed-form energy
fractions of nodal data built from chosen Legendre modes.
"""
import ctypes
import os

import numpy as np

from .cfl import cfl_number  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EQ_SW1D, EQ_SW2D, EQ_MHD2D, EQ_LINADV1D, EQ_VARADV1D, EQ_JINXIN1D = 1, 2, 3, 4, 5, 6
NVARS = {EQ_SW1D: 3, EQ_SW2D: 4, EQ_MHD2D: 9, EQ_LINADV1D: 1, EQ_VARADV1D: 2, EQ_JINXIN1D: 2}
DIMS = {EQ_SW1D: 1, EQ_SW2D: 2, EQ_MHD2D: 2, EQ_LINADV1D: 1, EQ_VARADV1D: 1, EQ_JINXIN1D: 1}
NCONSTR = {EQ_SW1D: 1, EQ_SW2D: 1, EQ_MHD2D: 2, EQ_LINADV1D: 0, EQ_VARADV1D: 0, EQ_JINXIN1D: 0}
IMEX_HT112, IMEX_SSP3 = 1, 2

FLAG_ALG2, FLAG_LOW_INADM, FLAG_ALG1, FLAG_NONFINITE, FLAG_ALG1_GUARD = 1, 2, 4, 8, 16


class OraCfg(ctypes.Structure):
    _fields_ = [
        ("eq", ctypes.c_int32), ("N", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lo", ctypes.c_double * 2), ("hi", ctypes.c_double * 2),
        ("gamma", ctypes.c_double), ("gravity", ctypes.c_double),
        ("cs", ctypes.c_double), ("cfl", ctypes.c_double),
        ("blending", ctypes.c_int32),
        ("alpha_max", ctypes.c_double), ("alpha_min", ctypes.c_double), ("alpha_force", ctypes.c_double),
        ("gll", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("ghost", ctypes.c_void_p),
        ("imex", ctypes.c_int32),
        ("relax_a", ctypes.c_double), ("relax_eps", ctypes.c_double),
        ("relax_l", ctypes.c_double), ("relax_q", ctypes.c_double),
        ("alw", ctypes.c_int32),
        ("threads", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        _lib = ctypes.CDLL(_LIBPATH)
    return _lib


def _p(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


BC_PERIODIC, BC_OUTFLOW, BC_WALL, BC_DIRICHLET = 0, 1, 2, 3


def make_cfg(eq, N, nx, ny=1, lo=(0.0, 0.0), hi=(1.0, 1.0), gamma=5.0 / 3.0, gravity=9.81, cs=0.9,
             cfl=None, blending=2, alpha_max=0.5, alpha_min=1e-3, alpha_force=-1.0, gll=False,
             bc=(0, 0, 0, 0), imex=0, relax=(3.0, 1e-2, 0.0, 1.0), alw=False, threads=1):
    """gll: Gauss-Lobatto-Legendre solution points with the g_2 correction (App. B)
    instead of Gauss-Legendre points with the Radau correction.
    bc: boundary kinds of the sides (x lo, x hi, y lo, y hi), BC_* (periodic by
    default); BC_DIRICHLET data go with each call (`ghost=` of step).
    imex: IMEX pair (IMEX_HT112, IMEX_SSP3) in place of the degree's explicit
    tableau; required by systems with a source.  relax: Jin-Xin (a, eps, l, q),
    f(u) = l u + q u^2/2 (Burgers by default).
    alw: time averages by the approximate Lax-Wendroff procedure (finite
    differences in time along Taylor states) instead of the cRK stages.
    cfl=None takes the Fourier limit of the scheme these select.
    threads: OpenMP threads of the element and face loops (the results are the
    same bits for any count)."""
    c = OraCfg()
    c.eq, c.N, c.nx, c.ny = eq, N, nx, (ny if DIMS[eq] == 2 else 1)
    c.lo[0], c.lo[1] = lo
    c.hi[0], c.hi[1] = hi
    c.gamma, c.gravity, c.cs = gamma, gravity, cs
    c.cfl = cfl_number(N, gll, imex) if cfl is None else cfl
    c.blending, c.alpha_max, c.alpha_min, c.alpha_force = blending, alpha_max, alpha_min, alpha_force
    c.gll = 1 if gll else 0
    for i in range(4):
        c.bc[i] = bc[i]
    c.ghost = None
    c.imex = imex
    c.relax_a, c.relax_eps, c.relax_l, c.relax_q = relax
    c.alw = 1 if alw else 0
    c.threads = threads
    return c


def shape(c):
    n1 = c.N + 1
    P = n1 if DIMS[c.eq] == 1 else n1 * n1
    return (NVARS[c.eq], c.nx * c.ny, P)


def nfp(c):
    return 1 if DIMS[c.eq] == 1 else c.N + 1


def refel(N, gll=False):
    n1 = N + 1
    out = {k: np.zeros(n1) for k in ("xi", "w", "VL", "VR", "gLp", "gRp")}
    D = np.zeros((n1, n1))
    Leg = np.zeros((n1, n1))
    rc = lib().ora_refel(N, 1 if gll else 0, _p(out["xi"]), _p(out["w"]), _p(D), _p(out["VL"]), _p(out["VR"]),
                         _p(out["gLp"]), _p(out["gRp"]), _p(Leg))
    assert rc == 0
    out["D"], out["Leg"] = D, Leg
    return out


def tableau(N):
    s = ctypes.c_int(0)
    A = np.zeros(36)
    b = np.zeros(6)
    assert lib().ora_tableau(N, ctypes.byref(s), _p(A), _p(b)) == 0
    n = s.value
    return A[: n * n].reshape(n, n).copy(), b[:n].copy()


def tableau_imex(imex):
    """(A~, b~, A, b) of IMEX pair imex: explicit and implicit parts."""
    s = ctypes.c_int(0)
    A, b, Ai, bi = np.zeros(36), np.zeros(6), np.zeros(36), np.zeros(6)
    assert lib().ora_tableau_imex(imex, ctypes.byref(s), _p(A), _p(b), _p(Ai), _p(bi)) == 0
    n = s.value
    return A[: n * n].reshape(n, n).copy(), b[:n].copy(), Ai[: n * n].reshape(n, n).copy(), bi[:n].copy()


def jinxin(what, u, a=3.0, eps=1e-2, c=0.0, l=0.0, q=1.0):
    """Jin-Xin pointwise parts: what in {'flux', 'source', 'implicit'} ('implicit': the
    solution x of x - c s(x) = u)."""
    code = {"flux": 0, "source": 1, "implicit": 2}[what]
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(2)
    assert lib().ora_jinxin(code, ctypes.c_double(a), ctypes.c_double(eps), ctypes.c_double(l), ctypes.c_double(q),
                            ctypes.c_double(c), _p(u), _p(out)) == 0
    return out


def physics(eq, what, d, u, w=None, gamma=5.0 / 3.0, gravity=9.81, ch=0.0):
    """Pointwise physics of one state: what in {'flux','nc','sigma','constraints','indicator','speeds'}."""
    code = {"flux": 0, "nc": 1, "sigma": 2, "constraints": 3, "indicator": 4, "speeds": 5}[what]
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(max(NVARS[eq], 2))
    rc = lib().ora_physics(eq, ctypes.c_double(gamma), ctypes.c_double(gravity), ctypes.c_double(ch), code, d,
                           _p(u), _p(w), _p(out))
    assert rc == 0
    n = {0: NVARS[eq], 1: NVARS[eq], 2: 1, 3: NCONSTR[eq], 4: 1, 5: 2}[code]
    return out[:n]


def ncols(eq, d):
    """Columns of B_d the oracle treats as not identically zero."""
    out = np.zeros(16, dtype=np.int32)
    n = lib().ora_ncols(eq, d, _p(out, ctypes.c_int))
    assert n >= 0
    return sorted(out[:n].tolist())


def dt_ch(c, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(2)
    assert lib().ora_dt_ch(ctypes.byref(c), _p(u), _p(out)) == 0
    return float(out[0]), float(out[1])


def alpha(c, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = c.nx * c.ny
    araw, al, tie = np.zeros(E), np.zeros(E), np.zeros(E, dtype=np.uint8)
    assert lib().ora_alpha(ctypes.byref(c), _p(u), _p(araw), _p(al), _p(tie, ctypes.c_uint8)) == 0
    return araw, al, tie


def step(c, u, dt=0.0, ch=-1.0, alpha_in=None, ghost=None):
    """One step.  dt > 0 is used as given, otherwise eq. time.step.2d; ch >= 0 overrides c_h;
    alpha_in replaces the indicator's blending coefficients; ghost holds the data of
    BC_DIRICHLET sides (layout of Config::ghost in oracle/scheme.hpp)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    gbuf = None if ghost is None else np.ascontiguousarray(ghost, dtype=np.float64)
    c.ghost = None if gbuf is None else gbuf.ctypes.data
    E = c.nx * c.ny
    d = DIMS[c.eq]
    out = {
        "u": np.zeros_like(u),
        "dt_ch": np.zeros(2),
        "alpha": np.zeros(E),
        "flags": np.zeros(E, dtype=np.uint32),
        "tie": np.zeros(E, dtype=np.uint8),
        "theta_face": np.ones((d, E, nfp(c))),
        "theta_elem": np.ones(E),
    }
    ain = None if alpha_in is None else np.ascontiguousarray(alpha_in, dtype=np.float64)
    rc = lib().ora_step(ctypes.byref(c), _p(u), _p(out["u"]), ctypes.c_double(dt), ctypes.c_double(ch), _p(ain),
                        _p(out["dt_ch"]), _p(out["alpha"]), _p(out["flags"], ctypes.c_uint32),
                        _p(out["tie"], ctypes.c_uint8), _p(out["theta_face"]), _p(out["theta_elem"]))
    c.ghost = None
    assert rc == 0, rc
    out["dt"], out["ch"] = float(out["dt_ch"][0]), float(out["dt_ch"][1])
    return out


def ghost_size(c):
    """Doubles of the BC_DIRICHLET data of configuration c: for each side b = 2 d + s
    (x lo, x hi[, y lo, y hi]) a block [quantity 3][variable M][face point along the side]."""
    M = NVARS[c.eq]
    tot = 0
    for d in range(DIMS[c.eq]):
        lines = c.ny if d == 0 else c.nx
        tot += 2 * 3 * M * lines * nfp(c)
    return tot


def time_averages(c, u, dt, ch=0.0):
    """(F [d][v][e][p], U, B^loc) of the element-local stage (or approximate LW) procedure."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    d = DIMS[c.eq]
    F = np.zeros((d,) + u.shape)
    U, Bl = np.zeros_like(u), np.zeros_like(u)
    assert lib().ora_time_averages(ctypes.byref(c), _p(u), ctypes.c_double(dt), ctypes.c_double(ch), _p(F), _p(U),
                                   _p(Bl)) == 0
    return F, U, Bl


def residual(c, u, dt, mode, ch=-1.0):
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    R = np.zeros_like(u)
    assert lib().ora_residual(ctypes.byref(c), _p(u), ctypes.c_double(dt), ctypes.c_double(ch), mode, _p(R)) == 0
    return R


def jvp(c, u, v, dt, ch):
    """J v of the step with dt, c_h, alpha and every theta frozen at their values at u."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(shape(c))
    un, Jv = np.zeros_like(u), np.zeros_like(u)
    assert lib().ora_jvp(ctypes.byref(c), _p(u), _p(v), ctypes.c_double(dt), ctypes.c_double(ch), _p(un),
                         _p(Jv)) == 0
    return un, Jv


def count_ops(c, u, dt, ch):
    """Operation counts [phase][add, mul, div, sqrt, exp] for phases (stage loop, face traces,
    faces, update, means with dt / c_h / indicator); counted serially (threads is ignored)."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    counts = np.zeros(25, dtype=np.uint64)
    threads = c.threads
    c.threads = 1
    try:
        rc = lib().ora_count_ops(ctypes.byref(c), _p(u), ctypes.c_double(dt), ctypes.c_double(ch),
                                 _p(counts, ctypes.c_uint64))
    finally:
        c.threads = threads
    assert rc == 0
    return counts.reshape(5, 5)


def step_parts(c, u, dt=0.0, ch=-1.0):
    """u^{n+1}, the lower order update u^L and the blend u* before Algorithm 2, the
    Algorithm 2 theta product per element and the flags, for one step as `step`."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    E = c.nx * c.ny
    out = {"u": np.zeros_like(u), "uL": np.zeros_like(u), "ustar": np.zeros_like(u), "theta_elem": np.ones(E),
           "flags": np.zeros(E, dtype=np.uint32)}
    rc = lib().ora_step_parts(ctypes.byref(c), _p(u), ctypes.c_double(dt), ctypes.c_double(ch), _p(out["u"]),
                              _p(out["uL"]), _p(out["ustar"]), _p(out["theta_elem"]),
                              _p(out["flags"], ctypes.c_uint32))
    assert rc == 0, rc
    return out


def face(c, d, side_m, side_p, af, dt, ch=0.0):
    """One face (Algorithm 1 with cfg blending = 2) from side data [a, F, U, s, si]
    (each M values: face u^n, traces of F_d and U, u^n at the node next to the face
    and the one after it).  Returns (F^-, F^+, theta product, guard)."""
    M = NVARS[c.eq]
    sm = np.ascontiguousarray(side_m, dtype=np.float64).reshape(5 * M)
    sp = np.ascontiguousarray(side_p, dtype=np.float64).reshape(5 * M)
    Fm, Fp = np.zeros(M), np.zeros(M)
    th = ctypes.c_double(1.0)
    g = ctypes.c_uint8(0)
    rc = lib().ora_face(ctypes.byref(c), d, _p(sm), _p(sp), ctypes.c_double(af), ctypes.c_double(dt),
                        ctypes.c_double(ch), _p(Fm), _p(Fp), ctypes.byref(th), ctypes.byref(g))
    assert rc == 0, rc
    return Fm, Fp, th.value, g.value


def vjp(c, u, lam, dt, ch, threads=0):
    """J^T lam of the step with dt, c_h, alpha and every theta frozen at their values at u
    (reverse mode, oracle/reverse.hpp); threads <= 0: the OpenMP default."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape(c))
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(shape(c))
    mu = np.zeros_like(u)
    rc = lib().ora_vjp(ctypes.byref(c), _p(u), _p(lam), ctypes.c_double(dt), ctypes.c_double(ch), _p(mu),
                       ctypes.c_int(threads))
    assert rc == 0, rc
    return mu


def run(c, u0, nsteps, save_at=()):
    """The oracle's own run of nsteps steps from u0 (dt from eq. time.step.2d each step):
    {k: state before step k for k in save_at (k = nsteps: the final state)}, and the
    (nsteps, 2) array of each step's (dt, c_h)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(shape(c))
    save_at = sorted(set(int(k) for k in save_at))
    saved = np.zeros((len(save_at),) + u0.shape)
    at = np.array(save_at, dtype=np.int32)
    dtch = np.zeros((nsteps, 2))
    rc = lib().ora_run(ctypes.byref(c), _p(u0), int(nsteps), len(save_at), _p(at, ctypes.c_int32), _p(saved),
                       _p(dtch))
    assert rc == 0, rc
    return {k: saved[i] for i, k in enumerate(save_at)}, dtch
