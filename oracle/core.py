"""ctypes wrapper around the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))

MODELS = {"orbit": 0, "eikonal": 1, "crown": 2}
SEARCH_MODES = {"table": 0, "scan_golden": 1, "seeded": 2, "table_walk": 3}
INTEGRATORS = {"euler": 0, "heun": 1}
KIND_FREE, KIND_TARGET, KIND_INACTIVE = 0, 1, 2


class ProblemStruct(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 4),
        ("lo", C.c_double * 4),
        ("hi", C.c_double * 4),
        ("model", C.c_int32),
        ("mu", C.c_double),
        ("accel", C.c_double),
        ("mdot", C.c_double),
        ("dt", C.c_double),
        ("lam", C.c_double),
        ("w_time", C.c_double),
        ("w_fuel", C.c_double),
        ("M", C.c_double),
        ("speed", C.c_double),
        ("tgt_c", C.c_double * 4),
        ("tgt_w", C.c_double * 4),
        ("integrator", C.c_int32),
        ("el_beta", C.c_double),
        ("el_gamma", C.c_double),
        ("el_a", C.c_double),
        ("el_e", C.c_double),
        ("el_omega", C.c_double),
    ]


class SearchStruct(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_angles", C.c_int32), ("n_scan", C.c_int32),
                ("n_golden", C.c_int32), ("n_local", C.c_int32), ("local_half_width", C.c_double),
                ("fallback_tol", C.c_double)]


def problem_struct(p):
    s = ProblemStruct()
    s.n[:] = [int(v) for v in p["n"]]
    s.lo[:] = [float(v) for v in p["lo"]]
    s.hi[:] = [float(v) for v in p["hi"]]
    s.model = MODELS[p["model"]]
    for f in ("mu", "accel", "mdot", "dt", "lam", "w_time", "w_fuel", "M", "speed"):
        setattr(s, f, float(p[f]))
    s.tgt_c[:] = [float(v) for v in p["tgt_c"]]
    s.tgt_w[:] = [float(v) for v in p["tgt_w"]]
    s.integrator = INTEGRATORS[p.get("integrator", "euler")]
    for f in ("el_beta", "el_gamma", "el_a", "el_e", "el_omega"):
        setattr(s, f, float(p.get(f, 0.0)))
    return s


def search_struct(sr):
    s = SearchStruct()
    s.mode = SEARCH_MODES[sr["mode"]]
    s.n_angles = int(sr.get("n_angles", 0))
    s.n_scan = int(sr.get("n_scan", 0))
    s.n_golden = int(sr.get("n_golden", 0))
    s.n_local = int(sr.get("n_local", 0))
    s.local_half_width = float(sr.get("local_half_width", 0.0))
    s.fallback_tol = float(sr.get("fallback_tol", 0.0))
    return s


_LIBS = {}


def load(precision="f64"):
    """Load (building first if needed) the oracle library."""
    if precision in _LIBS:
        return _LIBS[precision]
    lib64, lib32 = _build.LIB64, _build.LIB32
    path = lib64 if precision == "f64" else lib32
    src_m = os.path.getmtime(_build.SRC)
    if not os.path.exists(path) or os.path.getmtime(path) < src_m:
        _build.build(force=True)
    lib = C.CDLL(path)
    P = C.POINTER(ProblemStruct)
    S = C.POINTER(SearchStruct)
    vp = C.c_void_p
    i64 = C.c_int64
    lib.or_classify.argtypes = [P, vp, vp]
    lib.or_init_value.argtypes = [P, vp, vp]
    real = C.c_double if precision == "f64" else C.c_float
    lib.or_step.argtypes = [P, vp, C.c_int, real, real, vp]
    lib.or_interp.argtypes = [P, vp, vp]
    lib.or_interp.restype = real
    lib.or_interp_weights.argtypes = [P, vp, vp, vp]
    lib.or_interp_weights.restype = C.c_int
    lib.or_value_at.argtypes = [P, vp, vp]
    lib.or_value_at.restype = C.c_double
    lib.or_q.argtypes = [P, vp, i64, C.c_int, real]
    lib.or_q.restype = real
    lib.or_q_many.argtypes = [P, vp, vp, vp, vp, i64, vp]
    lib.or_residual.argtypes = [i64, vp, vp, vp, vp]
    lib.or_bellman_sweep.argtypes = [P, vp, S, vp, vp, vp, vp, vp]
    lib.or_bellman_nodes.argtypes = [P, vp, S, vp, vp, i64, vp, vp, vp, vp]
    lib.or_bellman_sweep_seeded.argtypes = [P, vp, S, vp, vp, vp, vp, vp, vp, vp]
    lib.or_bellman_sweep_walk.argtypes = [P, vp, S, vp, vp, vp, vp, vp, vp, vp]
    lib.or_policy_eval_sweep.argtypes = [P, vp, vp, vp, vp, vp]
    lib.or_solve_vi.argtypes = [P, vp, S, vp, vp, vp, C.c_double, C.c_double, i64, vp]
    lib.or_solve_vi.restype = i64
    lib.or_solve_pi.argtypes = [P, vp, S, vp, vp, vp, C.c_double, C.c_double, C.c_int32, i64,
                                vp, vp]
    lib.or_solve_pi.restype = i64
    lib.or_feedback.argtypes = [P, S, vp, vp, i64, C.c_double, vp, vp, vp, vp]
    lib.or_brute_thrust_min.argtypes = [P, vp, i64, i64, vp]
    lib.or_brute_thrust_min.restype = real
    lib.or_mask_from_coarse.argtypes = [P, vp, P, C.c_double, vp, vp]
    lib.or_rk4_step.argtypes = [P, vp, C.c_int, real, real, real]
    lib.or_policy_system.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.or_q_state.argtypes = [P, vp, vp, C.c_int, real, real]
    lib.or_q_state.restype = real
    lib.or_simulate.argtypes = [P, S, vp, vp, i64, C.c_double, C.c_int32, C.c_int32, C.c_double, vp, vp, vp]
    lib.or_running_cost.argtypes = [P, vp, C.c_int]
    lib.or_running_cost.restype = real
    lib.or_elements.argtypes = [P, vp, vp]
    lib.or_real_size.restype = C.c_int32
    lib._real = real
    lib._np_real = np.float64 if precision == "f64" else np.float32
    assert lib.or_real_size() == (8 if precision == "f64" else 4)
    _LIBS[precision] = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Oracle:
    """One problem instance on the oracle.  Arrays are numpy, C order [m][v_t][v_r][r]."""

    def __init__(self, problem, mask=None, precision="f64"):
        self.problem = problem
        self.lib = load(precision)
        self.dtype = self.lib._np_real
        self.ps = problem_struct(problem)
        self.ss = search_struct(problem["search"])
        n = problem["n"]
        self.shape = (n[3], n[2], n[1], n[0])
        self.N = int(np.prod(self.shape))
        self.mask = None
        if mask is not None:
            self.mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(self.shape))
        self.kind = np.zeros(self.shape, dtype=np.uint8)
        self.lib.or_classify(C.byref(self.ps), _ptr(self.mask), _ptr(self.kind))

    def _arr(self, V):
        return np.ascontiguousarray(np.asarray(V, dtype=self.dtype).reshape(self.shape))

    def init_value(self):
        V = np.empty(self.shape, dtype=self.dtype)
        self.lib.or_init_value(C.byref(self.ps), _ptr(self.kind), _ptr(V))
        return V

    def step(self, x, thr, u, tau=None):
        x = np.ascontiguousarray(np.asarray(x, dtype=self.dtype))
        z = np.empty(4, dtype=self.dtype)
        tau = self.problem["dt"] if tau is None else tau
        self.lib.or_step(C.byref(self.ps), _ptr(x), int(thr), u, tau, _ptr(z))
        return z

    def running_cost(self, x, thr):
        x = np.ascontiguousarray(np.asarray(x, dtype=self.dtype))
        return float(self.lib.or_running_cost(C.byref(self.ps), _ptr(x), int(thr)))

    def elements(self, x):
        """(a, e cos omega, e sin omega) of a crown-problem state."""
        x = np.ascontiguousarray(np.asarray(x, dtype=self.dtype))
        out = np.zeros(3, dtype=self.dtype)
        self.lib.or_elements(C.byref(self.ps), _ptr(x), _ptr(out))
        return out

    def interp(self, V, s):
        V = self._arr(V)
        s = np.ascontiguousarray(np.asarray(s, dtype=self.dtype))
        return float(self.lib.or_interp(C.byref(self.ps), _ptr(V), _ptr(s)))

    def interp_weights(self, s):
        s = np.ascontiguousarray(np.asarray(s, dtype=self.dtype))
        idx = np.zeros(16, dtype=np.int64)
        w = np.zeros(16, dtype=self.dtype)
        ok = self.lib.or_interp_weights(C.byref(self.ps), _ptr(s), _ptr(idx), _ptr(w))
        return bool(ok), idx, w

    def value_at(self, V, x):
        V = self._arr(V)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        return float(self.lib.or_value_at(C.byref(self.ps), _ptr(V), _ptr(x)))

    def q(self, V, j, thr, u):
        V = self._arr(V)
        return float(self.lib.or_q(C.byref(self.ps), _ptr(V), int(j), int(thr), u))

    def q_many(self, V, nodes, thr, ang):
        V = self._arr(V)
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64).reshape(-1))
        thr = np.ascontiguousarray(np.asarray(thr, dtype=np.uint8).reshape(-1))
        ang = np.ascontiguousarray(np.asarray(ang, dtype=self.dtype).reshape(-1))
        out = np.empty(nodes.size, dtype=self.dtype)
        self.lib.or_q_many(C.byref(self.ps), _ptr(V), _ptr(nodes), _ptr(thr), _ptr(ang), nodes.size,
                           _ptr(out))
        return out

    def residual(self, Vold, Vnew):
        Vo, Vn = self._arr(Vold), self._arr(Vnew)
        out = np.zeros(3, dtype=np.float64)
        self.lib.or_residual(self.N, _ptr(self.kind), _ptr(Vo), _ptr(Vn), _ptr(out))
        return dict(max_rel=out[0], sum_abs=out[1], max_abs=out[2])

    def bellman_sweep(self, V, search=None):
        Vin = self._arr(V)
        ss = self.ss if search is None else search_struct(search)
        Vout = np.empty_like(Vin)
        ang = np.empty_like(Vin)
        thr = np.empty(self.shape, dtype=np.uint8)
        margin = np.empty_like(Vin)
        self.lib.or_bellman_sweep(C.byref(self.ps), _ptr(self.kind), C.byref(ss), _ptr(Vin),
                                  _ptr(Vout), _ptr(ang), _ptr(thr), _ptr(margin))
        return Vout, ang, thr, margin

    def bellman_sweep_seeded(self, V, seed, search=None):
        """Seeded sweep; returns V, angle, throttle, margin and the fallback flags."""
        Vin = self._arr(V)
        sd = self._arr(seed)
        ss = self.ss if search is None else search_struct(search)
        Vout = np.empty_like(Vin)
        ang = np.empty_like(Vin)
        thr = np.empty(self.shape, dtype=np.uint8)
        margin = np.empty_like(Vin)
        fb = np.empty(self.shape, dtype=np.uint8)
        self.lib.or_bellman_sweep_seeded(C.byref(self.ps), _ptr(self.kind), C.byref(ss), _ptr(Vin), _ptr(sd),
                                         _ptr(Vout), _ptr(ang), _ptr(thr), _ptr(margin), _ptr(fb))
        return Vout, ang, thr, margin, fb

    def bellman_sweep_walk(self, V, ang_prev, search=None):
        """Sweep with the table walk from the angles ang_prev (None: the full
        table); returns V, angle, throttle, margin and the thrust evaluations."""
        Vin = self._arr(V)
        prev = None if ang_prev is None else self._arr(ang_prev)
        ss = self.ss if search is None else search_struct(search)
        Vout = np.empty_like(Vin)
        ang = np.empty_like(Vin)
        thr = np.empty(self.shape, dtype=np.uint8)
        margin = np.empty_like(Vin)
        ev = np.zeros(1, dtype=np.int64)
        self.lib.or_bellman_sweep_walk(C.byref(self.ps), _ptr(self.kind), C.byref(ss), _ptr(Vin), _ptr(prev),
                                       _ptr(Vout), _ptr(ang), _ptr(thr), _ptr(margin), _ptr(ev))
        return Vout, ang, thr, margin, int(ev[0])

    def bellman_nodes(self, V, nodes, search=None):
        Vin = self._arr(V)
        ss = self.ss if search is None else search_struct(search)
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64))
        cnt = nodes.size
        kind_at = np.ascontiguousarray(self.kind.reshape(-1)[nodes])
        Vout = np.empty(cnt, dtype=self.dtype)
        ang = np.empty(cnt, dtype=self.dtype)
        thr = np.empty(cnt, dtype=np.uint8)
        margin = np.empty(cnt, dtype=self.dtype)
        self.lib.or_bellman_nodes(C.byref(self.ps), _ptr(kind_at), C.byref(ss), _ptr(Vin),
                                  _ptr(nodes), cnt, _ptr(Vout), _ptr(ang), _ptr(thr),
                                  _ptr(margin))
        return Vout, ang, thr, margin

    def policy_eval_sweep(self, V, ang, thr):
        Vin = self._arr(V)
        a = self._arr(ang)
        t = np.ascontiguousarray(np.asarray(thr, dtype=np.uint8).reshape(self.shape))
        Vout = np.empty_like(Vin)
        self.lib.or_policy_eval_sweep(C.byref(self.ps), _ptr(self.kind), _ptr(Vin), _ptr(Vout),
                                      _ptr(a), _ptr(t))
        return Vout

    def solve_vi(self, V0=None, tol_abs=1e-8, tol_rel=0.0, max_sweeps=100000, search=None):
        V = self.init_value() if V0 is None else self._arr(V0).copy()
        ss = self.ss if search is None else search_struct(search)
        ang = np.zeros(self.shape, dtype=self.dtype)
        thr = np.zeros(self.shape, dtype=np.uint8)
        res = np.zeros(3, dtype=np.float64)
        k = self.lib.or_solve_vi(C.byref(self.ps), _ptr(self.kind), C.byref(ss), _ptr(V),
                                 _ptr(ang), _ptr(thr), tol_abs, tol_rel, max_sweeps, _ptr(res))
        return dict(V=V, angle=ang, thr=thr, sweeps=int(k), converged=k > 0,
                    resid=dict(max_rel=res[0], sum_abs=res[1], max_abs=res[2]))

    def solve_pi(self, V0=None, tol_abs=1e-8, tol_rel=0.0, eval_sweeps=20, max_outer=100000,
                 search=None):
        V = self.init_value() if V0 is None else self._arr(V0).copy()
        ss = self.ss if search is None else search_struct(search)
        ang = np.zeros(self.shape, dtype=self.dtype)
        thr = np.zeros(self.shape, dtype=np.uint8)
        res = np.zeros(3, dtype=np.float64)
        ev = np.zeros(1, dtype=np.int64)
        k = self.lib.or_solve_pi(C.byref(self.ps), _ptr(self.kind), C.byref(ss), _ptr(V),
                                 _ptr(ang), _ptr(thr), tol_abs, tol_rel, int(eval_sweeps),
                                 max_outer, _ptr(res), _ptr(ev))
        return dict(V=V, angle=ang, thr=thr, outer=int(k), converged=k > 0,
                    eval_sweeps=int(ev[0]),
                    resid=dict(max_rel=res[0], sum_abs=res[1], max_abs=res[2]))

    def feedback(self, V, states, tau=None, search=None, with_margin=False):
        """eq:feed at arbitrary states: angle, throttle and Q of the chosen
        control per state, and with with_margin the search's tie margin."""
        Vin = self._arr(V)
        ss = self.ss if search is None else search_struct(search)
        st = np.ascontiguousarray(np.asarray(states, dtype=np.float64).reshape(-1, 4))
        cnt = st.shape[0]
        ang = np.empty(cnt, dtype=self.dtype)
        thr = np.empty(cnt, dtype=np.uint8)
        q = np.empty(cnt, dtype=self.dtype)
        tau = self.problem["dt"] if tau is None else tau
        margin = np.empty(cnt, dtype=self.dtype)
        self.lib.or_feedback(C.byref(self.ps), C.byref(ss), _ptr(Vin), _ptr(st), cnt,
                             float(tau), _ptr(ang), _ptr(thr), _ptr(q), _ptr(margin))
        if with_margin:
            return ang, thr, q, margin
        return ang, thr, q

    def q_state(self, V, y, thr, u, tau=None):
        """Q of the control (thr, u) at an arbitrary state y (eq:feed's argument)."""
        Vin = self._arr(V)
        y = np.ascontiguousarray(np.asarray(y, dtype=self.dtype))
        tau = self.problem["dt"] if tau is None else tau
        return float(self.lib.or_q_state(C.byref(self.ps), _ptr(Vin), _ptr(y), int(thr), u, tau))

    def policy_evaluate_exact(self, V, ang, thr):
        """Exact policy evaluation (eq:p_eval as a linear system, Section 3):
        the sparse system assembled from the Q1 weights and solved by a
        direct sparse factorisation; fixed nodes keep V's values."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spl
        Vf = self._arr(V)
        a = self._arr(ang)
        t = np.ascontiguousarray(np.asarray(thr, dtype=np.uint8).reshape(self.shape))
        free = (self.kind.reshape(-1) == KIND_FREE)
        nf = int(free.sum())
        unknown = np.full(self.N, -1, dtype=np.int64)
        unknown[free] = np.arange(nf)
        rows = np.zeros(17 * max(nf, 1), dtype=np.int64)
        cols = np.zeros_like(rows)
        vals = np.zeros(17 * max(nf, 1))
        rhs = np.zeros(max(nf, 1))
        nnz = np.zeros(1, dtype=np.int64)
        self.lib.or_policy_system(C.byref(self.ps), _ptr(self.kind), _ptr(Vf), _ptr(a), _ptr(t), _ptr(unknown),
                                  _ptr(rows), _ptr(cols), _ptr(vals), _ptr(rhs), _ptr(nnz))
        k = int(nnz[0])
        A = sp.csr_matrix((vals[:k], (rows[:k], cols[:k])), shape=(nf, nf))
        v = spl.spsolve(A.tocsc(), rhs[:nf])
        out = np.array(Vf, dtype=np.float64).reshape(-1)
        out[free] = v
        return out.reshape(self.shape)

    def rk4_step(self, x, thr, u, h, drag=0.0):
        x = np.ascontiguousarray(np.asarray(x, dtype=self.dtype)).copy()
        self.lib.or_rk4_step(C.byref(self.ps), _ptr(x), int(thr), u, h, drag)
        return x

    def simulate(self, V, states, tau, steps, substeps=1, search=None, history=True, drag=0.0):
        """Closed loop from states (count x 4): returns final states and, with
        history, the trajectory ((steps+1) x count x 4) and the controls.
        drag: Example 2's drag coefficient on the simulated system only."""
        Vin = self._arr(V)
        ss = self.ss if search is None else search_struct(search)
        st = np.ascontiguousarray(np.asarray(states, dtype=np.float64).reshape(-1, 4)).copy()
        cnt = st.shape[0]
        traj = np.zeros((steps + 1, cnt, 4)) if history else None
        thr = np.zeros((steps, cnt), dtype=np.uint8) if history else None
        ang = np.zeros((steps, cnt), dtype=self.dtype) if history else None
        self.lib.or_simulate(C.byref(self.ps), C.byref(ss), _ptr(Vin), _ptr(st), cnt, float(tau), int(steps),
                             int(substeps), float(drag), _ptr(traj), _ptr(thr), _ptr(ang))
        return st, traj, thr, ang

    def brute_thrust_min(self, V, j, n_angles):
        Vin = self._arr(V)
        u = np.zeros(1, dtype=self.dtype)
        q = self.lib.or_brute_thrust_min(C.byref(self.ps), _ptr(Vin), int(j), int(n_angles),
                                         _ptr(u))
        return float(q), float(u[0])

    def node_coords(self, j):
        """Physical coordinates of flat node j (plain grid definition; the
        crown problem's theta axis has h = (hi - lo)/n)."""
        n = self.problem["n"]
        i = []
        for k in range(4):
            i.append(j % n[k])
            j //= n[k]
        lo, hi = self.problem["lo"], self.problem["hi"]
        per = self.problem["model"] == "crown"
        h = [(hi[k] - lo[k]) / (n[k] if (per and k == 3) else n[k] - 1) for k in range(4)]
        return np.array([lo[k] + i[k] * h[k] for k in range(4)])


def mask_from_coarse(coarse_problem, Vc, fine_problem, dilate, thresh=None):
    lib = load("f64")
    pc, pf = problem_struct(coarse_problem), problem_struct(fine_problem)
    Vc = np.ascontiguousarray(np.asarray(Vc, dtype=np.float64))
    n = fine_problem["n"]
    mask = np.zeros((n[3], n[2], n[1], n[0]), dtype=np.uint8)
    dil = np.ascontiguousarray(np.asarray(dilate, dtype=np.int32))
    if thresh is None:
        thresh = 0.5 * coarse_problem["M"]
    lib.or_mask_from_coarse(C.byref(pc), _ptr(Vc), C.byref(pf), float(thresh), _ptr(dil),
                            _ptr(mask))
    return mask
