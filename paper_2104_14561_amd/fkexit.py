"""Python binding of libfkexit (include/fkexit.h): argument marshalling only.

Every step of the backward pass runs in the library's HIP kernels; PyTorch
provides device memory (the workspace and the outputs) and the stream.  The
binding refuses to run when the HIP library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FKEXIT_LIB names another build of the same library (the AddressSanitizer
# build of the host code, for instance)
LIB_PATH = os.environ.get("FKEXIT_LIB") or os.path.join(_HERE, "libfkexit.so")

FK_OK = 0
STATUS = {0: "FK_OK", -1: "FK_ERR_ARG", -2: "FK_ERR_UNSUPPORTED", -3: "FK_ERR_WORKSPACE",
          -4: "FK_ERR_HIP", -5: "FK_ERR_NONFINITE", -6: "FK_ERR_STATE"}
COEF = {"const": 0, "cellular2d": 1, "abc3d": 2, "rolls2d": 3, "runaway3d": 4}
FACE = {"exit1": 0, "exit0": 1, "reflect": 2}
REGION = {"box": 0, "ball": 1}
PREC = {"f64": 0, "f32": 1}
FORM = {"fused": 0, "ell": 1}
HERMITE = {"r1": 0, "r2": 1}
STEP_KERNEL = {"auto": 0, "node": 1, "group": 2, "split": 3, "box": 4}
MAX_THETA = 8

EXPORTED = ["fk_last_error", "fk_version", "fk_gh_rule", "fk_plan_create", "fk_plan_destroy",
            "fk_plan_get_info", "fk_plan_layout", "fk_plan_set_workspace", "fk_forward",
            "fk_forward_from", "fk_forward_horizons", "fk_forward_static", "fk_step", "fk_apply_step", "fk_export_cells", "fk_export_ell",
            "fk_check_flags", "fk_adjoint", "fk_profile_pass", "fk_profile_adjoint", "fk_tune",
            "fk_probe_precision", "fk_probe_lds_atomics"]


class FkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Axis(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nodes", ctypes.POINTER(ctypes.c_double)),
                ("periodic", ctypes.c_int)]


class _Problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("ax", _Axis * 3), ("coef_kind", ctypes.c_int),
                ("coef", ctypes.c_double * 16), ("D", ctypes.c_double),
                ("region_kind", ctypes.c_int), ("center", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("gh_q", ctypes.c_int), ("dt", ctypes.c_double),
                ("n_steps", ctypes.c_int), ("t0", ctypes.c_double),
                ("force_f64", ctypes.c_int), ("face", (ctypes.c_int * 2) * 3)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("form", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("ckpt_every", ctypes.c_int), ("block", ctypes.c_int),
                ("step_kernel", ctypes.c_int), ("columns", ctypes.c_int),
                ("hermite", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int), ("d", ctypes.c_int), ("gh_q", ctypes.c_int),
                ("n_quad", ctypes.c_int), ("n_steps", ctypes.c_int), ("n_theta", ctypes.c_int),
                ("n_nodes", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("ell_width", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
                ("ell_entries", ctypes.c_int64), ("adj_point_nodes", ctypes.c_int64),
                ("adj_box_nodes", ctypes.c_int64)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("step_kernel", ctypes.c_int), ("ms_per_step", ctypes.c_double * 5)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfkexit.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "fk_last_error": (ctypes.c_char_p, []),
        "fk_version": (ctypes.c_int, []),
        "fk_gh_rule": (ctypes.c_int, [ctypes.c_int, dp, dp]),
        "fk_plan_create": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int,
                                          ctypes.POINTER(_Options), PP]),
        "fk_plan_destroy": (None, [vp]),
        "fk_plan_get_info": (ctypes.c_int, [vp, ctypes.POINTER(_Info)]),
        "fk_plan_layout": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]),
        "fk_plan_set_workspace": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "fk_forward": (ctypes.c_int, [vp, ip, ctypes.c_int, vp, vp]),
        "fk_forward_from": (ctypes.c_int, [vp, vp, ctypes.c_int, ip, ctypes.c_int, vp, vp]),
        "fk_forward_static": (ctypes.c_int, [vp, ip, ctypes.c_int, vp, vp]),
        "fk_forward_horizons": (ctypes.c_int, [vp, ip, ctypes.c_int, vp, vp]),
        "fk_step": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "fk_apply_step": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "fk_export_cells": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "fk_export_ell": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp]),
        "fk_check_flags": (ctypes.c_int, [vp, vp, ip]),
        "fk_adjoint": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fk_profile_pass": (ctypes.c_int, [vp, dp, ip, vp]),
        "fk_profile_adjoint": (ctypes.c_int, [vp, vp, vp, dp, ip, vp]),
        "fk_tune": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(_Options),
                                   ctypes.c_int, vp, ctypes.c_size_t, vp,
                                   ctypes.POINTER(_TuneResult)]),
        "fk_probe_lds_atomics": (ctypes.c_int, [ctypes.c_int, dp, vp, ctypes.c_size_t, vp]),
        "fk_probe_precision": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.c_int,
                                              ctypes.POINTER(_Options), ctypes.c_double, vp,
                                              ctypes.c_double, vp, ctypes.c_size_t, vp,
                                              ctypes.POINTER(ctypes.c_size_t), ip, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != FK_OK:
        raise FkError(status, load().fk_last_error().decode())


def gh_rule(q: int):
    """The library's own Gauss-Hermite rule (host computation)."""
    a = np.zeros(q)
    w = np.zeros(q)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load().fk_gh_rule(q, a.ctypes.data_as(dp), w.ctypes.data_as(dp)))
    return a, w


def _marshal(problems, force_f64=None) -> tuple:
    arr = (_Problem * len(problems))()
    keep = []
    for i, pr in enumerate(problems):
        s = arr[i]
        s.d = pr.d
        for a in range(3):
            if a < pr.d:
                nodes = np.ascontiguousarray(pr.axes[a].nodes, dtype=np.float64)
                keep.append(nodes)
                s.ax[a].n = nodes.shape[0]
                s.ax[a].nodes = nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                s.ax[a].periodic = int(pr.axes[a].periodic)
        s.coef_kind = COEF[pr.coef_kind]
        for k, v in enumerate(pr.coef):
            s.coef[k] = float(v)
        s.D = float(pr.D)
        s.region_kind = REGION[pr.region_kind]
        for k in range(min(3, len(pr.center))):
            s.center[k] = float(pr.center[k])
        s.radius = float(pr.radius)
        s.gh_q = int(pr.gh_q)
        s.dt = float(pr.dt)
        s.n_steps = int(pr.n_steps)
        s.t0 = float(pr.t0)
        s.force_f64 = int(bool(force_f64[i])) if force_f64 is not None else 0
        faces = getattr(pr, "faces", None)
        for a in range(3):
            for side in range(2):
                s.face[a][side] = FACE[faces[a][side]] if faces and a < len(faces) else 0
    return arr, keep


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


class Plan:
    """A plan over one or more problem instances (batched, uneven grids).

    precision: "f64" or "f32" (FP64 landing points and cells, FP32 weights,
    gathers, accumulation and fields); form: "fused" or "ell"; use_graph:
    capture the N-step loop once and replay it; ckpt_every: adjoint checkpoint
    interval (0 = no adjoint).  step_kernel: "auto", "node", "group", "split",
    "box", or "tune" (fk_tune times the layouts on this device first and the
    plan takes the fastest; the choice and timings are in .tuned).
    allocate=False builds the plan on the host only (for its info: workspace
    size, node counts); calls need a workspace.  force_f64: per-instance
    flags (an FP32 plan computes the flagged instances in FP64; see
    precision_probe).  columns: columns per launch of the assembled
    product in forward_horizons (1..4).  hermite: "r1" (values and first
    derivatives) or "r2" (also the mixed derivatives; d <= 2, fused form,
    forward calls).
    """

    def __init__(self, problems, precision: str = "f64", form: str = "fused",
                 use_graph: bool = False, ckpt_every: int = 0, device: str = "cuda",
                 step_kernel: str = "auto", allocate: bool = True, force_f64=None,
                 columns: int = 1, hermite: str = "r1"):
        import torch
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.tuned = None
        if step_kernel == "tune":
            self.tuned = tune(self.problems, precision=precision, form=form,
                              use_graph=use_graph, device=device)
            step_kernel = self.tuned["step_kernel"]
        lib = load()
        self.force_f64 = None if force_f64 is None else [bool(v) for v in force_f64]
        arr, keep = _marshal(self.problems, self.force_f64)
        opt = _Options()
        opt.precision = PREC[precision]
        opt.form = FORM[form]
        opt.use_graph = int(bool(use_graph))
        opt.ckpt_every = int(ckpt_every)
        opt.step_kernel = STEP_KERNEL[step_kernel]
        opt.columns = int(columns)
        opt.hermite = HERMITE[hermite]
        h = ctypes.c_void_p()
        _check(lib.fk_plan_create(arr, len(self.problems), ctypes.byref(opt), ctypes.byref(h)))
        del keep
        self._h = h
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        info = _Info()
        _check(lib.fk_plan_get_info(h, ctypes.byref(info)))
        self.info = info
        n = len(self.problems)
        off = (ctypes.c_int64 * (n + 1))()
        cnt = (ctypes.c_int64 * n)()
        _check(lib.fk_plan_layout(h, off, cnt))
        self.node_offset = [int(v) for v in off]
        self.active_count = [int(v) for v in cnt]
        self.device = torch.device(device)
        self.workspace = None
        if not allocate:
            return
        nbytes = max(int(info.workspace_bytes), 256)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = _ptr(self.workspace)
        aligned = (base + 255) // 256 * 256
        _check(lib.fk_plan_set_workspace(h, ctypes.c_void_p(aligned), nbytes,
                                         ctypes.c_void_p(_stream())))

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            load().fk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout helpers -----------------------------------------------------
    @property
    def n_nodes(self) -> int:
        return int(self.info.n_nodes)

    @property
    def n_theta(self) -> int:
        return int(self.info.n_theta)

    def split(self, field):
        """Views of a packed field (last dim = all nodes) per instance, shaped
        to each instance's grid."""
        out = []
        for i, pr in enumerate(self.problems):
            a, b = self.node_offset[i], self.node_offset[i + 1]
            out.append(field[..., a:b].reshape(field.shape[:-1] + pr.shape))
        return out

    def pack(self, fields: Sequence):
        import torch
        return torch.cat([f.reshape(-1) for f in fields]).to(self.device, self.dtype).contiguous()

    # -- calls --------------------------------------------------------------
    def forward(self, snaps: Sequence[int] = (0,), stream=None):
        import torch
        sn = np.ascontiguousarray(snaps, dtype=np.int32)
        out = torch.empty((len(sn), self.n_nodes), dtype=self.dtype, device=self.device)
        _check(load().fk_forward(self._h, sn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 len(sn), ctypes.c_void_p(_ptr(out)),
                                 ctypes.c_void_p(_stream(stream))))
        return out

    def forward_horizons(self, horizons: Sequence[int], stream=None):
        """fk_forward_horizons (Algorithm 1): one field per horizon m (in steps
        from t0), the exit probability by t0 + m dt; [len(horizons), n_nodes]."""
        import torch
        hz = np.ascontiguousarray(horizons, dtype=np.int32)
        out = torch.empty((len(hz), self.n_nodes), dtype=self.dtype, device=self.device)
        _check(load().fk_forward_horizons(self._h, hz.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                          len(hz), ctypes.c_void_p(_ptr(out)),
                                          ctypes.c_void_p(_stream(stream))))
        return out

    def forward_static(self, snaps: Sequence[int] = (0,), stream=None):
        """fk_forward_static: the backward pass on the library's static
        device buffer (no workspace needed; see include/fkexit.h)."""
        import torch
        sn = np.ascontiguousarray(snaps, dtype=np.int32)
        out = torch.empty((len(sn), self.n_nodes), dtype=self.dtype, device=self.device)
        _check(load().fk_forward_static(self._h, sn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                        len(sn), ctypes.c_void_p(_ptr(out)),
                                        ctypes.c_void_p(_stream(stream))))
        return out

    def forward_from(self, u_start, start_step: int, snaps: Sequence[int] = (0,), stream=None):
        import torch
        u_start = u_start.to(self.device, self.dtype).contiguous()
        sn = np.ascontiguousarray(snaps, dtype=np.int32)
        out = torch.empty((len(sn), self.n_nodes), dtype=self.dtype, device=self.device)
        _check(load().fk_forward_from(self._h, ctypes.c_void_p(_ptr(u_start)), int(start_step),
                                      sn.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(sn),
                                      ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_stream(stream))))
        return out

    def step(self, n: int, u_next, stream=None):
        import torch
        u_next = u_next.to(self.device, self.dtype).contiguous()
        out = torch.empty(self.n_nodes, dtype=self.dtype, device=self.device)
        _check(load().fk_step(self._h, int(n), ctypes.c_void_p(_ptr(u_next)),
                              ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_stream(stream))))
        return out

    def apply_step(self, n: int, x, transpose: bool = False, stream=None):
        """fk_apply_step: A_n x for x = (d + 1) packed fields [u; g_0; ..]
        (shape [d + 1, n_nodes]) -> one field, or A_n^T x for one field x ->
        [d + 1, n_nodes] (transpose=True)."""
        import torch
        d = int(self.info.d)
        x = x.to(self.device, self.dtype).contiguous()
        if transpose:
            out = torch.empty((d + 1, self.n_nodes), dtype=self.dtype, device=self.device)
        else:
            out = torch.empty(self.n_nodes, dtype=self.dtype, device=self.device)
        _check(load().fk_apply_step(self._h, int(n), int(bool(transpose)),
                                    ctypes.c_void_p(_ptr(x)), ctypes.c_void_p(_ptr(out)),
                                    ctypes.c_void_p(_stream(stream))))
        return out

    def export_cells(self, inst: int, n: int, stream=None):
        import torch
        Ja = self.active_count[inst]
        d, Q = int(self.info.d), int(self.info.n_quad)
        cells = torch.empty((max(Ja, 1), Q, d), dtype=torch.int32, device=self.device)
        exitf = torch.empty((max(Ja, 1), Q), dtype=torch.uint8, device=self.device)
        _check(load().fk_export_cells(self._h, int(inst), int(n), ctypes.c_void_p(_ptr(cells)),
                                      ctypes.c_void_p(_ptr(exitf)), ctypes.c_void_p(_stream(stream))))
        return cells[:Ja], exitf[:Ja]

    def export_ell(self, n: int, stream=None):
        import torch
        na, W = int(self.info.n_active), int(self.info.ell_width)
        cols = torch.empty((W, na), dtype=torch.int32, device=self.device)
        vals = torch.empty((W, na), dtype=self.dtype, device=self.device)
        em = torch.empty(max(na, 1), dtype=self.dtype, device=self.device)
        _check(load().fk_export_ell(self._h, int(n), ctypes.c_void_p(_ptr(cols)),
                                    ctypes.c_void_p(_ptr(vals)), ctypes.c_void_p(_ptr(em)),
                                    ctypes.c_void_p(_stream(stream))))
        return cols, vals, em[:na]

    def check_flags(self, stream=None) -> int:
        f = ctypes.c_int(0)
        st = load().fk_check_flags(self._h, ctypes.c_void_p(_stream(stream)), ctypes.byref(f))
        _check(st)
        return int(f.value)

    def profile_pass(self, stream=None):
        """Mean per-launch durations (ms) of the slope pass, fused step, ELL
        assembly and ELL product over one pass, timed with HIP events."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int * 4)()
        _check(load().fk_profile_pass(self._h, ms, cnt, ctypes.c_void_p(_stream(stream))))
        names = ("slopes", "step_fused", "assemble_ell", "ell_apply")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(names)}

    def adjoint(self, lam0, stream=None):
        """Gradient of <lam0, u^0> w.r.t. theta per instance, and dJ/du^N."""
        import torch
        lam0 = lam0.to(self.device, self.dtype).contiguous()
        grad = torch.zeros((len(self.problems), MAX_THETA), dtype=torch.float64, device=self.device)
        lamN = torch.empty(self.n_nodes, dtype=self.dtype, device=self.device)
        _check(load().fk_adjoint(self._h, ctypes.c_void_p(_ptr(lam0)), ctypes.c_void_p(_ptr(grad)),
                                 ctypes.c_void_p(_ptr(lamN)), ctypes.c_void_p(_stream(stream))))
        return grad[:, : self.n_theta], lamN

    def profile_adjoint(self, lam0, stream=None):
        """Mean per-step durations (ms) of the adjoint's kernel groups (slope
        pass, transposed step per landing point, transposed slopes + fold,
        recomputed forward step, transposed step in box form) over one
        fk_adjoint call, timed with HIP events."""
        import torch
        lam0 = lam0.to(self.device, self.dtype).contiguous()
        grad = torch.zeros((len(self.problems), MAX_THETA), dtype=torch.float64, device=self.device)
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int * 5)()
        _check(load().fk_profile_adjoint(self._h, ctypes.c_void_p(_ptr(lam0)),
                                         ctypes.c_void_p(_ptr(grad)), ms, cnt,
                                         ctypes.c_void_p(_stream(stream))))
        names = ("slopes", "adjoint_step", "slopes_T", "recompute_step", "adjoint_box")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(names)}


def tune(problems, precision: str = "f64", form: str = "fused", use_graph: bool = False,
         trial_steps: int = 16, device: str = "cuda", stream=None):
    """fk_tune: time every step layout on a trial_steps-step copy of the
    problems and return {"step_kernel": name, "ms_per_step": {name: ms}}."""
    import torch
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    probe = Plan(problems, precision=precision, form=form, use_graph=use_graph, device=device,
                 allocate=False)
    nbytes = int(probe.info.workspace_bytes) * 5 // 4 + (1 << 20)
    probe.close()
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
    aligned = (_ptr(ws) + 255) // 256 * 256
    arr, keep = _marshal(list(problems))
    opt = _Options()
    opt.precision = PREC[precision]
    opt.form = FORM[form]
    opt.use_graph = int(bool(use_graph))
    res = _TuneResult()
    _check(load().fk_tune(arr, len(problems), ctypes.byref(opt), int(trial_steps),
                          ctypes.c_void_p(aligned), nbytes, ctypes.c_void_p(_stream(stream)),
                          ctypes.byref(res)))
    del keep, ws
    names = {v: k for k, v in STEP_KERNEL.items()}
    return {"step_kernel": names[res.step_kernel],
            "ms_per_step": {names[k]: float(res.ms_per_step[k]) for k in range(1, 5)
                            if res.ms_per_step[k] > 0}}


def precision_probe(problems, tol: float = 1e-5, lam0=None, grad_tol: float = 1e-4,
                    use_graph: bool = False, step_kernel: str = "auto", device: str = "cuda",
                    stream=None):
    """fk_probe_precision: per instance, max |u^0 (FP64) - u^0 (FP32)| over
    one backward pass of each and, with a cotangent lam0 (packed field),
    the relative gradient difference of the two adjoints; flags
    (diff > tol / 2 or grad diff > grad_tol / 2) for
    Plan(..., force_f64=flags).  Returns (flags, diffs, grad_diffs)."""
    import torch
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    lib = load()
    arr, keep = _marshal(list(problems))
    opt = _Options()
    opt.use_graph = int(bool(use_graph))
    opt.step_kernel = STEP_KERNEL[step_kernel]
    need = ctypes.c_size_t(0)
    n = len(problems)
    flags = (ctypes.c_int * n)()
    diffs = (ctypes.c_double * n)()
    gdiffs = (ctypes.c_double * n)()
    _check(lib.fk_probe_precision(arr, n, ctypes.byref(opt), float(tol), None, float(grad_tol),
                                  None, 0, None, ctypes.byref(need), flags, diffs, gdiffs))
    lam = None
    if lam0 is not None:
        lam = lam0.to(torch.device(device), torch.float64).contiguous()
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=torch.device(device))
    aligned = (_ptr(ws) + 255) // 256 * 256
    _check(lib.fk_probe_precision(arr, n, ctypes.byref(opt), float(tol),
                                  ctypes.c_void_p(_ptr(lam)) if lam is not None else None,
                                  float(grad_tol), ctypes.c_void_p(aligned), int(need.value),
                                  ctypes.c_void_p(_stream(stream)), None, flags, diffs, gdiffs))
    del keep, ws
    return ([bool(v) for v in flags], [float(v) for v in diffs],
            [float(v) for v in gdiffs] if lam0 is not None else None)


def probe_lds_atomics(f32: bool = False, device: str = "cuda", stream=None) -> float:
    """fk_probe_lds_atomics: lane-level LDS atomic adds per second (FP64 or
    FP32, conflict-free addresses)."""
    import torch
    ws = torch.empty(2048, dtype=torch.float64, device=torch.device(device))
    rate = ctypes.c_double(0.0)
    _check(load().fk_probe_lds_atomics(int(bool(f32)), ctypes.byref(rate), ctypes.c_void_p(_ptr(ws)),
                                       2048 * 8, ctypes.c_void_p(_stream(stream))))
    return float(rate.value)


def solve(problems, snaps: Sequence[int] = (0,), **plan_kw):
    """Backward pass; returns per-instance tensors [len(snaps)] + grid shape."""
    plan = Plan(problems, **plan_kw)
    out = plan.forward(snaps)
    res = plan.split(out)
    plan.close()
    return res
