"""Thin Python binding of libdpo.so (the C ABI in include/dpo.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
libdpo.  PyTorch supplies device memory (contiguous CUDA tensors on ROCm) and
the current stream.  If the library is missing the import fails loudly; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpo.so")

DPO_OK, DPO_ENOCONV, DPO_EINVAL, DPO_ENOMEM, DPO_EHIP, DPO_ENUMERIC = 0, 1, -1, -2, -3, -4
MODELS = {"orbit": 0, "eikonal": 1, "crown": 2}
SEARCH = {"table": 0, "scan_golden": 1, "seeded": 2, "table_walk": 3}
INTEGRATORS = {"euler": 0, "heun": 1}
KIND_FREE, KIND_TARGET, KIND_INACTIVE = 0, 1, 2


class DpoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdpo error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 4), ("lo", C.c_double * 4), ("hi", C.c_double * 4)]


class Problem(C.Structure):
    _fields_ = [("model", C.c_int32), ("mu", C.c_double), ("accel", C.c_double), ("mdot", C.c_double),
                ("dt", C.c_double), ("lam", C.c_double), ("w_time", C.c_double), ("w_fuel", C.c_double),
                ("M", C.c_double), ("speed", C.c_double), ("tgt_c", C.c_double * 4),
                ("tgt_w", C.c_double * 4), ("integrator", C.c_int32), ("el_beta", C.c_double),
                ("el_gamma", C.c_double), ("el_a", C.c_double), ("el_e", C.c_double), ("el_omega", C.c_double)]


class Search(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_angles", C.c_int32), ("n_scan", C.c_int32),
                ("n_golden", C.c_int32), ("n_local", C.c_int32), ("local_half_width", C.c_double),
                ("fallback_tol", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("resid_max_rel", C.c_double), ("resid_sum_abs", C.c_double),
                ("resid_max_abs", C.c_double), ("converged", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("eval_sweeps", C.c_int64), ("evals", C.c_int64),
                ("fallback_nodes", C.c_int64), ("verify_steps", C.c_int64), ("resid_max_rel", C.c_double),
                ("resid_sum_abs", C.c_double), ("resid_max_abs", C.c_double), ("seconds", C.c_double),
                ("stalled", C.c_int32), ("converged", C.c_int32), ("greedy_seconds", C.c_double),
                ("eval_seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libdpo.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdpo.so not built at {LIB_PATH}: run `python -m paper_2407_14675_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sig = {
        "dpo_create": [C.POINTER(Grid), C.POINTER(Problem), C.POINTER(Search), vp, C.POINTER(vp)],
        "dpo_destroy": [vp],
        "dpo_last_error": [vp],
        "dpo_sizes": [vp, C.POINTER(i64), C.POINTER(i64)],
        "dpo_get_kind": [vp, vp, vp],
        "dpo_set_search": [vp, C.POINTER(Search)],
        "dpo_set_kernel_path": [vp, i32],
        "dpo_kernel_path": [vp],
        "dpo_eval_sweep_bytes": [vp, C.POINTER(i64)],
        "dpo_init_value": [vp, vp, vp],
        "dpo_bellman_sweep": [vp, vp, vp, vp, vp, vp, vp],
        "dpo_bellman_sweep_seeded": [vp, vp, vp, vp, vp, vp, vp, vp],
        "dpo_policy_eval_sweep": [vp, vp, vp, vp, vp, vp, vp],
        "dpo_policy_eval_sweep_last": [vp, vp, vp, vp],
        "dpo_policy_eval_sweep_static": [vp, vp, vp, vp, vp, vp, vp],
        "dpo_set_eval_path": [vp, i32],
        "dpo_eval_path": [vp],
        "dpo_solve_vi": [vp, vp, vp, vp, dbl, i64, i32, C.POINTER(Stats), vp],
        "dpo_solve_pi": [vp, vp, vp, vp, dbl, i32, i64, vp, C.POINTER(Stats), vp],
        "dpo_policy_evaluate": [vp, vp, vp, vp, dbl, i32, C.POINTER(i64), C.POINTER(dbl), vp],
        "dpo_value_at": [vp, vp, vp, vp, vp],
        "dpo_extract_feedback": [vp, vp, vp, i64, dbl, vp, vp, vp, vp],
        "dpo_simulate": [vp, vp, vp, i64, dbl, i32, i32, dbl, vp, vp, vp, vp],
        "dpo_mask_from_coarse": [vp, vp, C.POINTER(Grid), dbl, vp, vp, vp],
        "dpo_probe_interp": [vp, vp, vp, i64, vp, vp],
        "dpo_probe_q": [vp, vp, vp, vp, vp, i64, vp, vp],
        "dpo_probe_foot": [vp, vp, vp, vp, i64, vp, vp],
        "dpo_set_block": [vp, i32],
        "dpo_batch_create": [i32, vp, vp, C.POINTER(Search), C.POINTER(vp)],
        "dpo_batch_destroy": [vp],
        "dpo_batch_last_error": [vp],
        "dpo_batch_sizes": [vp, vp, vp],
        "dpo_batch_init_value": [vp, vp, vp],
        "dpo_batch_solve_vi": [vp, vp, vp, vp, dbl, i64, i32, i32, vp, vp, vp],
        "dpo_batch_solve_sequential": [vp, vp, vp, vp, dbl, i64, i32, vp, vp, vp],
        "dpo_batch_time_config": [vp, i32, i32, i32, vp],
        "dpo_mlp_create": [vp, C.POINTER(vp)],
        "dpo_mlp_destroy": [vp],
        "dpo_mlp_last_error": [vp],
        "dpo_mlp_set_params": [vp, vp],
        "dpo_mlp_get_params": [vp, vp],
        "dpo_mlp_get_grad": [vp, vp],
        "dpo_mlp_set_adam": [vp, dbl, dbl, dbl, dbl],
        "dpo_mlp_steps": [vp],
        "dpo_mlp_forward": [vp, vp, i64, vp, vp],
        "dpo_mlp_grad": [vp, vp, vp, i64, vp, vp, vp],
        "dpo_mlp_train": [vp, vp, vp, i64, vp, i32, vp, vp],
        "dpo_mlp_propose": [vp, vp, vp, vp],
        "dpo_feasible_nodes": [vp, vp, dbl, vp, C.POINTER(i64), vp],
        "dpo_gather_pairs": [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp],
        "dpo_probe_copy": [vp, vp, i64, vp],
        "dpo_probe_read": [vp, i64, vp, vp],
        "dpo_probe_fma": [i32, i32, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.dpo_destroy.restype = None
    lib.dpo_last_error.restype = C.c_char_p
    lib.dpo_batch_destroy.restype = None
    lib.dpo_batch_last_error.restype = C.c_char_p
    lib.dpo_mlp_destroy.restype = None
    lib.dpo_mlp_last_error.restype = C.c_char_p
    lib.dpo_mlp_steps.restype = C.c_int64
    _lib = lib
    return lib


def grid_struct(problem):
    g = Grid()
    g.n[:] = [int(v) for v in problem["n"]]
    g.lo[:] = [float(v) for v in problem["lo"]]
    g.hi[:] = [float(v) for v in problem["hi"]]
    return g


def problem_struct(problem):
    p = Problem()
    p.model = MODELS[problem["model"]]
    for f in ("mu", "accel", "mdot", "dt", "lam", "w_time", "w_fuel", "M", "speed"):
        setattr(p, f, float(problem[f]))
    p.tgt_c[:] = [float(v) for v in problem["tgt_c"]]
    p.tgt_w[:] = [float(v) for v in problem["tgt_w"]]
    p.integrator = INTEGRATORS[problem.get("integrator", "euler")]
    for f in ("el_beta", "el_gamma", "el_a", "el_e", "el_omega"):
        setattr(p, f, float(problem.get(f, 0.0)))
    return p


def search_struct(search):
    s = Search()
    s.mode = SEARCH[search["mode"]]
    s.n_angles = int(search.get("n_angles", 0))
    s.n_scan = int(search.get("n_scan", 0))
    s.n_golden = int(search.get("n_golden", 0))
    s.n_local = int(search.get("n_local", 0))
    s.local_half_width = float(search.get("local_half_width", 0.0))
    s.fallback_tol = float(search.get("fallback_tol", 0.0))
    return s


def _p(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "libdpo needs contiguous device tensors"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Context:
    """One problem (grid + physics + search) on the device."""

    def __init__(self, problem, mask=None, device="cuda"):
        self.lib = load()
        self.problem = problem
        self.device = torch.device(device)
        n = problem["n"]
        self.shape = (n[3], n[2], n[1], n[0])
        self.N = n[0] * n[1] * n[2] * n[3]
        if mask is not None:
            mask = mask.to(self.device, torch.uint8).contiguous().reshape(-1)
            assert mask.numel() == self.N
        self._g, self._pr, self._s = grid_struct(problem), problem_struct(problem), search_struct(problem["search"])
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        rc = self.lib.dpo_create(C.byref(self._g), C.byref(self._pr), C.byref(self._s), _p(mask), C.byref(h))
        if rc != DPO_OK:
            raise DpoError(rc, self.lib.dpo_last_error(None).decode())
        self.h = h
        nn, nf = C.c_int64(), C.c_int64()
        self.lib.dpo_sizes(self.h, C.byref(nn), C.byref(nf))
        self.n_free = nf.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.dpo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(DPO_OK,)):
        if rc not in allow:
            raise DpoError(rc, self.lib.dpo_last_error(self.h).decode())
        return rc

    def _arr(self, t, dtype, name, n=None):
        """A node array (or n elements) of the given dtype, contiguous on the
        device: checked here, since the library cannot see a tensor's size."""
        if t is None:
            return None
        n = self.N if n is None else n
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype \
                or t.numel() != n:
            raise DpoError(DPO_EINVAL, f"{name} must be a contiguous device tensor of {n} {dtype} elements")
        return _p(t)

    def _v(self, t, name="V"):
        return self._arr(t, torch.float32, name)

    def _ang(self, t, name="pol_ang"):
        return self._arr(t, torch.float32, name)

    def _thr(self, t, name="pol_thr"):
        return self._arr(t, torch.uint8, name)

    def _res(self, t):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64 \
                or t.numel() < 5:
            raise DpoError(DPO_EINVAL, "resid must be a contiguous device float64 tensor of at least 5 elements")
        return _p(t)

    # ---------------------------------------------------------- buffers
    def empty_value(self):
        return torch.empty(self.shape, dtype=torch.float32, device=self.device)

    def empty_policy(self):
        return (torch.zeros(self.shape, dtype=torch.float32, device=self.device),
                torch.zeros(self.shape, dtype=torch.uint8, device=self.device))

    def set_kernel_path(self, path):
        """0 automatic, 1 direct 16-corner gathers, 2 factorised thrust kernel."""
        self._check(self.lib.dpo_set_kernel_path(self.h, int(path)))

    def set_eval_path(self, path):
        """Kernel of the policy-array evaluation sweeps: 0 automatic, 1 free
        list (descriptors inside policy iteration), 2 LDS value bricks."""
        self._check(self.lib.dpo_set_eval_path(self.h, int(path)))

    def eval_path(self):
        return self.lib.dpo_eval_path(self.h)

    def kernel_path(self):
        rc = self.lib.dpo_kernel_path(self.h)
        if rc < 0:
            raise DpoError(rc, self.lib.dpo_last_error(self.h).decode())
        return rc

    def eval_sweep_bytes(self):
        """Algorithmic bytes of one frozen-policy sweep from foot descriptors."""
        b = C.c_int64()
        self._check(self.lib.dpo_eval_sweep_bytes(self.h, C.byref(b)))
        return b.value

    def set_block(self, block):
        """Workgroup size of the factorised sweeps (64..512, multiple of 64)."""
        self._check(self.lib.dpo_set_block(self.h, int(block)))

    def set_search(self, search):
        self._s = search_struct(search)
        self._check(self.lib.dpo_set_search(self.h, C.byref(self._s)))

    def kind(self):
        k = torch.empty(self.shape, dtype=torch.uint8, device=self.device)
        self._check(self.lib.dpo_get_kind(self.h, _p(k), _stream()))
        return k

    def init_value(self, V=None):
        V = self.empty_value() if V is None else V
        self._check(self.lib.dpo_init_value(self.h, self._v(V), _stream()))
        return V

    # ------------------------------------------------------------ sweeps
    def bellman_sweep(self, V_in, V_out, pol_ang=None, pol_thr=None, resid=None):
        return self._check(self.lib.dpo_bellman_sweep(self.h, self._v(V_in, "V_in"), self._v(V_out, "V_out"),
                                                       self._ang(pol_ang), self._thr(pol_thr), self._res(resid),
                                                       _stream()))

    def bellman_sweep_seeded(self, V_in, V_out, pol_ang, pol_thr, seed, resid=None):
        return self._check(self.lib.dpo_bellman_sweep_seeded(self.h, self._v(V_in, "V_in"), self._v(V_out, "V_out"),
                                                              self._ang(pol_ang), self._thr(pol_thr),
                                                              self._ang(seed, "seed"), self._res(resid), _stream()))

    def policy_eval_sweep(self, V_in, V_out, pol_ang, pol_thr, resid=None):
        return self._check(self.lib.dpo_policy_eval_sweep(self.h, self._v(V_in, "V_in"), self._v(V_out, "V_out"),
                                                           self._ang(pol_ang), self._thr(pol_thr), self._res(resid),
                                                           _stream()))

    def policy_eval_sweep_static(self, V_in, V_out, pol_ang, pol_thr, resid=None):
        """policy_eval_sweep with its scratch in the library's static device
        array: the call allocates nothing."""
        return self._check(self.lib.dpo_policy_eval_sweep_static(self.h, self._v(V_in, "V_in"),
                                                                  self._v(V_out, "V_out"), self._ang(pol_ang),
                                                                  self._thr(pol_thr), self._res(resid), _stream()))

    def policy_eval_sweep_last(self, V_in, V_out):
        """Frozen-policy sweep for the policy of the last Bellman sweep."""
        return self._check(self.lib.dpo_policy_eval_sweep_last(self.h, self._v(V_in, "V_in"), self._v(V_out, "V_out"),
                                                                _stream()))

    # ----------------------------------------------------------- solvers
    def solve_vi(self, V, pol_ang, pol_thr, tol_rel=1e-6, max_sweeps=100000, check_every=16):
        st = Stats()
        rc = self.lib.dpo_solve_vi(self.h, self._v(V), self._ang(pol_ang), self._thr(pol_thr), float(tol_rel),
                                   int(max_sweeps),
                                   int(check_every), C.byref(st), _stream())
        self._check(rc, allow=(DPO_OK, DPO_ENOCONV))
        return rc, st.as_dict()

    def solve_pi(self, V, pol_ang, pol_thr, tol_rel=1e-6, eval_sweeps=20, max_outer=100000, seed=None):
        st = Stats()
        rc = self.lib.dpo_solve_pi(self.h, self._v(V), self._ang(pol_ang), self._thr(pol_thr), float(tol_rel),
                                   int(eval_sweeps), int(max_outer), self._ang(seed, "seed"), C.byref(st), _stream())
        self._check(rc, allow=(DPO_OK, DPO_ENOCONV))
        return rc, st.as_dict()

    def policy_evaluate(self, V, pol_ang, pol_thr, tol_rel=1e-7, max_iter=500):
        """Exact policy evaluation by GMRES (V in/out); returns (rc, operator
        applications, final relative residual)."""
        mv = C.c_int64()
        rel = C.c_double()
        rc = self.lib.dpo_policy_evaluate(self.h, self._v(V), self._ang(pol_ang), self._thr(pol_thr), float(tol_rel),
                                          int(max_iter),
                                          C.byref(mv), C.byref(rel), _stream())
        self._check(rc, allow=(DPO_OK, DPO_ENOCONV))
        return rc, mv.value, rel.value

    # ------------------------------------------------- read-out / feedback
    def value_at(self, V, x):
        xs = (C.c_double * 4)(*[float(v) for v in x])
        out = C.c_double()
        self._check(self.lib.dpo_value_at(self.h, self._v(V), xs, C.byref(out), _stream()))
        return out.value

    def feedback(self, V, states, tau=None):
        states = torch.as_tensor(states, dtype=torch.float64).to(self.device).contiguous().reshape(-1, 4)
        n = states.shape[0]
        ang = torch.empty(n, dtype=torch.float32, device=self.device)
        thr = torch.empty(n, dtype=torch.uint8, device=self.device)
        q = torch.empty(n, dtype=torch.float32, device=self.device)
        tau = self.problem["dt"] if tau is None else tau
        self._check(self.lib.dpo_extract_feedback(self.h, self._v(V), _p(states), n, float(tau), _p(ang), _p(thr),
                                                  _p(q), _stream()))
        return ang, thr, q

    def simulate(self, V, states, tau=None, steps=1, substeps=1, history=True, drag=0.0):
        """Closed loop from states (n x 4): feedback, then RK4 with the control
        held, `steps` times; drag > 0 adds Example 2's drag to the simulated
        system only.  Returns the final states (device, float64) and, with
        history, the trajectory ((steps+1) x n x 4) and the controls
        (steps x n)."""
        st = torch.as_tensor(states, dtype=torch.float64).to(self.device).contiguous().reshape(-1, 4).clone()
        n = st.shape[0]
        traj = thr = ang = None
        if history:
            traj = torch.empty((steps + 1, n, 4), dtype=torch.float64, device=self.device)
            thr = torch.empty((steps, n), dtype=torch.uint8, device=self.device)
            ang = torch.empty((steps, n), dtype=torch.float32, device=self.device)
        tau = self.problem["dt"] if tau is None else tau
        self._check(self.lib.dpo_simulate(self.h, self._v(V), _p(st), n, float(tau), int(steps), int(substeps),
                                          float(drag), _p(traj), _p(thr), _p(ang), _stream()))
        return st, traj, thr, ang

    def mask_from_coarse(self, Vc, fine_problem, thresh, dilate):
        g = grid_struct(fine_problem)
        n = fine_problem["n"]
        mask = torch.empty((n[3], n[2], n[1], n[0]), dtype=torch.uint8, device=self.device)
        dil = (C.c_int32 * 4)(*[int(d) for d in dilate])
        self._check(self.lib.dpo_mask_from_coarse(self.h, self._v(Vc, "Vc"), C.byref(g), float(thresh), dil, _p(mask),
                                                  _stream()))
        return mask

    # -------------------------------------------- training pairs (network)
    def feasible_nodes(self, V, thresh):
        """Packed coordinates (int32 view of u32) of the free nodes with V < thresh, in node order."""
        nodes = torch.empty(max(1, self.n_free), dtype=torch.int32, device=self.device)
        n = C.c_int64()
        self._check(self.lib.dpo_feasible_nodes(self.h, self._v(V), float(thresh), _p(nodes), C.byref(n), _stream()))
        return nodes[: n.value]

    def gather_pairs(self, nodes, sel, pol_ang, pol_thr):
        """Inputs (n x 4, scaled positions) and targets (cos, sin, throttle, 0) at nodes[sel]."""
        import numpy as np

        sel = np.ascontiguousarray(sel, dtype=np.int32)
        n = sel.shape[0]
        x = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        tgt = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        self._check(self.lib.dpo_gather_pairs(self.h, _p(nodes), nodes.numel(), sel.ctypes.data_as(C.c_void_p), n,
                                              self._ang(pol_ang), self._thr(pol_thr), _p(x), _p(tgt), _stream()))
        return x, tgt

    # ------------------------------------------------------------ probes
    def probe_interp(self, V, pts):
        pts = torch.as_tensor(pts, dtype=torch.float32).to(self.device).contiguous().reshape(-1, 4)
        out = torch.empty(pts.shape[0], dtype=torch.float32, device=self.device)
        self._check(self.lib.dpo_probe_interp(self.h, self._v(V), _p(pts), pts.shape[0], _p(out), _stream()))
        return out

    def probe_q(self, V, nodes, thr, angle):
        nodes = torch.as_tensor(nodes, dtype=torch.int32).to(self.device).contiguous()
        thr = torch.as_tensor(thr, dtype=torch.uint8).to(self.device).contiguous()
        angle = torch.as_tensor(angle, dtype=torch.float32).to(self.device).contiguous()
        q = torch.empty(nodes.numel(), dtype=torch.float32, device=self.device)
        torch.cuda.synchronize(self.device)
        self._check(self.lib.dpo_probe_q(self.h, self._v(V), _p(nodes), _p(thr), _p(angle), nodes.numel(), _p(q),
                                         _stream()))
        return q

    def probe_foot(self, nodes, thr, angle):
        nodes = torch.as_tensor(nodes, dtype=torch.int32).to(self.device).contiguous()
        thr = torch.as_tensor(thr, dtype=torch.uint8).to(self.device).contiguous()
        angle = torch.as_tensor(angle, dtype=torch.float32).to(self.device).contiguous()
        off = torch.empty((nodes.numel(), 4), dtype=torch.float32, device=self.device)
        torch.cuda.synchronize(self.device)
        self._check(self.lib.dpo_probe_foot(self.h, _p(nodes), _p(thr), _p(angle), nodes.numel(), _p(off),
                                            _stream()))
        return off


def _ptr_array(tensors):
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else _p(t).value
    return arr


class Batch:
    """Many problems (own grid and physics, shared search) solved together by
    value iteration: one kernel launch per sweep for all running problems,
    S sweeps per hipGraph replay."""

    def __init__(self, problems, device="cuda"):
        self.lib = load()
        self.problems = list(problems)
        self.device = torch.device(device)
        n = len(self.problems)
        grids = (Grid * n)(*[grid_struct(p) for p in self.problems])
        probs = (Problem * n)(*[problem_struct(p) for p in self.problems])
        self._s = search_struct(self.problems[0]["search"])
        h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        rc = self.lib.dpo_batch_create(n, grids, probs, C.byref(self._s), C.byref(h))
        if rc != DPO_OK:
            raise DpoError(rc, self.lib.dpo_batch_last_error(None).decode())
        self.h = h
        self.n = n
        nn = (C.c_int64 * n)()
        nf = (C.c_int64 * n)()
        self.lib.dpo_batch_sizes(self.h, nn, nf)
        self.n_nodes = list(nn)
        self.n_free = list(nf)
        self.shapes = [(p["n"][3], p["n"][2], p["n"][1], p["n"][0]) for p in self.problems]

    def close(self):
        if getattr(self, "h", None):
            self.lib.dpo_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(DPO_OK,)):
        if rc not in allow:
            raise DpoError(rc, self.lib.dpo_batch_last_error(self.h).decode())
        return rc

    def _arrs(self, ts, dtype, name):
        """One node array per problem, each of its problem's size."""
        if ts is None:
            return None
        ts = list(ts)
        if len(ts) != self.n:
            raise DpoError(DPO_EINVAL, f"{name}: {self.n} arrays expected, got {len(ts)}")
        for t, shape in zip(ts, self.shapes):
            n = shape[0] * shape[1] * shape[2] * shape[3]
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype \
                    or t.numel() != n:
                raise DpoError(DPO_EINVAL, f"{name}: each must be a contiguous device tensor of its problem's "
                                           f"node count in {dtype}")
        return _ptr_array(ts)

    def init_values(self):
        Vs = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.shapes]
        self._check(self.lib.dpo_batch_init_value(self.h, _ptr_array(Vs), _stream()))
        return Vs

    def empty_policies(self):
        return ([torch.zeros(s, dtype=torch.float32, device=self.device) for s in self.shapes],
                [torch.zeros(s, dtype=torch.uint8, device=self.device) for s in self.shapes])

    def solve_vi(self, Vs, angs=None, thrs=None, tol_rel=1e-6, max_sweeps=100000, sweeps_per_graph=16, block=256):
        st = (BatchStats * self.n)()
        sec = C.c_double()
        rc = self.lib.dpo_batch_solve_vi(self.h, self._arrs(Vs, torch.float32, "Vs"),
                                         self._arrs(angs, torch.float32, "angs"),
                                         self._arrs(thrs, torch.uint8, "thrs"), float(tol_rel), int(max_sweeps),
                                         int(sweeps_per_graph), int(block), st, C.byref(sec), _stream())
        self._check(rc, allow=(DPO_OK, DPO_ENOCONV))
        return rc, [s.as_dict() for s in st], sec.value

    def solve_sequential(self, Vs, angs, thrs, tol_rel=1e-6, max_sweeps=100000, check_every=16):
        st = (BatchStats * self.n)()
        sec = C.c_double()
        rc = self.lib.dpo_batch_solve_sequential(self.h, self._arrs(Vs, torch.float32, "Vs"),
                                                 self._arrs(angs, torch.float32, "angs"),
                                                 self._arrs(thrs, torch.uint8, "thrs"),
                                                 float(tol_rel), int(max_sweeps), int(check_every), st,
                                                 C.byref(sec), _stream())
        self._check(rc, allow=(DPO_OK, DPO_ENOCONV))
        return rc, [s.as_dict() for s in st], sec.value

    def time_config(self, block, sweeps_per_graph, replays=2):
        out = C.c_double()
        self._check(self.lib.dpo_batch_time_config(self.h, int(block), int(sweeps_per_graph), int(replays),
                                                   C.byref(out)))
        return out.value


MLP_PARAMS = 17539


class Mlp:
    """The control-proposal network on the device (parameters, Adam state)."""

    def __init__(self, params=None, device="cuda"):
        import numpy as np

        self.lib = load()
        self.device = torch.device(device)
        h = C.c_void_p()
        buf = None
        if params is not None:
            buf = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
            assert buf.size == MLP_PARAMS
        torch.cuda.synchronize(self.device)
        rc = self.lib.dpo_mlp_create(None if buf is None else buf.ctypes.data_as(C.c_void_p), C.byref(h))
        if rc != DPO_OK:
            raise DpoError(rc, self.lib.dpo_mlp_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.dpo_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != DPO_OK:
            raise DpoError(rc, self.lib.dpo_mlp_last_error(self.h).decode())

    def params(self):
        import numpy as np

        out = np.empty(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.dpo_mlp_get_params(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, params):
        import numpy as np

        buf = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        assert buf.size == MLP_PARAMS
        self._check(self.lib.dpo_mlp_set_params(self.h, buf.ctypes.data_as(C.c_void_p)))

    def last_grad(self):
        import numpy as np

        out = np.empty(MLP_PARAMS, dtype=np.float32)
        self._check(self.lib.dpo_mlp_get_grad(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.dpo_mlp_set_adam(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def steps(self):
        return int(self.lib.dpo_mlp_steps(self.h))

    def forward(self, x):
        x = x.contiguous()
        y = torch.empty((x.shape[0], 3), dtype=torch.float32, device=self.device)
        self._check(self.lib.dpo_mlp_forward(self.h, _p(x), x.shape[0], _p(y), _stream()))
        return y

    def grad(self, x, tgt):
        """(gradient tensor, mean loss tensor) of the batch; parameters unchanged."""
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self._check(self.lib.dpo_mlp_grad(self.h, _p(x.contiguous()), _p(tgt.contiguous()), x.shape[0], _p(g),
                                          _p(loss), _stream()))
        return g, loss

    def train_epoch(self, x, tgt, perm=None, batch=4096):
        """One epoch of Adam steps; returns the per-batch loss tensor."""
        import numpy as np

        n = x.shape[0]
        steps = (n + batch - 1) // batch if batch > 0 else 1
        hist = torch.empty(max(1, steps), dtype=torch.float32, device=self.device)
        pp = None
        if perm is not None:
            perm = np.ascontiguousarray(perm, dtype=np.int32)
            assert perm.size == n
            pp = perm.ctypes.data_as(C.c_void_p)
        self._check(self.lib.dpo_mlp_train(self.h, _p(x.contiguous()), _p(tgt.contiguous()), n, pp, int(batch),
                                           _p(hist), _stream()))
        return hist

    def propose(self, ctx, seed=None):
        """Seed angles at every free node of ctx (float32, node-shaped; other nodes 0)."""
        if seed is None:
            seed = torch.zeros(ctx.shape, dtype=torch.float32, device=self.device)
        self._check(self.lib.dpo_mlp_propose(self.h, ctx.h, ctx._ang(seed, "seed"), _stream()))
        return seed


def _check_global(rc):
    if rc != DPO_OK:
        raise DpoError(rc, load().dpo_last_error(None).decode())
    return rc


def probe_copy(src, dst):
    """dst = src with the library's 16-byte streaming copy (float32 device
    tensors of equal size, a multiple of 4)."""
    return _check_global(load().dpo_probe_copy(_p(src), _p(dst), src.numel(), _stream()))


def probe_read(src, sink):
    """Stream src (float32 device tensor) through 16-byte loads."""
    return _check_global(load().dpo_probe_read(_p(src), src.numel(), _p(sink), _stream()))


def probe_fma(blocks, iters, sink):
    """blocks x 256 threads x iters x 8 plain FP32 fused multiply-adds."""
    return _check_global(load().dpo_probe_fma(int(blocks), int(iters), _p(sink), _stream()))
