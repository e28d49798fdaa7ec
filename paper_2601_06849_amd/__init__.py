"""Python binding of libetdds: the spectral ETD2RK-DS stepper for MI355X.

Argument marshalling only.  Every step of the method runs in the HIP kernels
of ``libetdds.so`` (built in-tree by ``paper_2601_06849_amd.build``); the
functions below carry the same names as the C entry points declared in
``include/etdds.h`` and take torch device tensors for the field and the
workspace.  There is no fallback: if the library is missing or was built
for another GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libetdds.so")

ETD_OK, ETD_EINVAL, ETD_EUNSUPPORTED, ETD_EWORKSPACE, ETD_EHIP, ETD_ENONFINITE = 0, -1, -2, -3, -4, -5
ETD_FP64, ETD_FP32, ETD_BF16X6, ETD_FP64_FP32, ETD_FP64_BF16X6 = 0, 1, 2, 3, 4

RXN = {"none": 0, "linear": 1, "fisher": 2, "allen_cahn": 3, "ac_mms": 4, "saturating": 5,
       "fhn_cubic": 6, "fhn_classic": 7}
PRECISION = {"fp64": ETD_FP64, "fp32": ETD_FP32, "bf16x6": ETD_BF16X6, "fp64_fp32": ETD_FP64_FP32,
             "fp64_bf16x6": ETD_FP64_BF16X6}
# precisions whose state (fields) is FP64
FP64_STATE = ("fp64", "fp64_fp32", "fp64_bf16x6")


class EtdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"etdds status {status}: {message}")
        self.status = status


class etd_problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("ncomp", ctypes.c_int),
        ("kappa", ctypes.c_double * 2),
        ("q", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("rxn", ctypes.c_int),
        ("rxn_param", ctypes.c_double * 8),
        ("pade", ctypes.c_int),
        ("precision", ctypes.c_int),
    ]


_lib = None

EXPORTS = ("etd_plan_create", "etd_plan_workspace_bytes", "etd_plan_upload", "etd_advance", "etd_compare",
           "etd_compare_noalloc",
           "etd_plan_problem", "etd_plan_table", "etd_timing_enable", "etd_timing_read",
           "etd_adjoint_workspace_bytes", "etd_adjoint_workspace_bytes_segment", "etd_adjoint",
           "etd_plan_tiles", "etd_plan_set_tiles", "etd_plan_autotune",
           "etd_plan_set_schedule", "etd_plan_schedule",
           "etd_batch_create", "etd_batch_workspace_bytes", "etd_batch_upload", "etd_batch_advance",
           "etd_batch_autotune", "etd_batch_tiles", "etd_batch_groups", "etd_batch_destroy",
           "etd_graph_capture", "etd_batch_graph_capture", "etd_graph_launch", "etd_graph_destroy",
           "etd_plan_destroy", "etd_status_string", "etd_last_error")


def lib():
    """Load libetdds.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2601_06849_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, dp, ip = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        ipp = ctypes.POINTER(ctypes.c_int)
        d = ctypes.c_double
        sig = {
            "etd_plan_create": [ctypes.POINTER(etd_problem), ctypes.POINTER(vp)],
            "etd_plan_workspace_bytes": [vp, ctypes.POINTER(sz)],
            "etd_plan_upload": [vp, vp, sz, vp],
            "etd_advance": [vp, vp, d, ip, vp, vp],
            "etd_compare": [vp, vp, vp, dp, vp, vp],
            "etd_compare_noalloc": [vp, vp, vp, vp, vp],
            "etd_plan_problem": [vp, ctypes.POINTER(etd_problem)],
            "etd_plan_table": [vp, ip, ip, ip, dp, sz],
            "etd_timing_enable": [vp, ip],
            "etd_timing_read": [vp, dp, ctypes.POINTER(ctypes.c_longlong)],
            "etd_adjoint_workspace_bytes": [vp, ip, ctypes.POINTER(sz)],
            "etd_adjoint_workspace_bytes_segment": [vp, ip, ip, ctypes.POINTER(sz)],
            "etd_adjoint": [vp, vp, d, ip, vp, vp, dp, vp, vp, sz, vp],
            "etd_plan_tiles": [vp, ipp],
            "etd_plan_set_tiles": [vp, ipp],
            "etd_plan_autotune": [vp, vp, vp],
            "etd_plan_set_schedule": [vp, ip],
            "etd_plan_schedule": [vp, ipp],
            "etd_batch_create": [ctypes.POINTER(etd_problem), ip, ctypes.POINTER(vp)],
            "etd_batch_workspace_bytes": [vp, ctypes.POINTER(sz)],
            "etd_batch_upload": [vp, vp, sz, vp],
            "etd_batch_advance": [vp, ctypes.POINTER(vp), d, ip, vp, vp],
            "etd_batch_autotune": [vp, vp, vp],
            "etd_batch_tiles": [vp, ip, ipp],
            "etd_batch_groups": [vp, ipp],
            "etd_batch_destroy": [vp],
            "etd_graph_capture": [vp, vp, d, ip, vp, vp, ctypes.POINTER(vp)],
            "etd_batch_graph_capture": [vp, ctypes.POINTER(vp), d, ip, vp, vp, ctypes.POINTER(vp)],
            "etd_graph_launch": [vp, vp],
            "etd_graph_destroy": [vp],
            "etd_plan_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ip
        L.etd_status_string.argtypes = [ip]
        L.etd_status_string.restype = ctypes.c_char_p
        L.etd_last_error.argtypes = []
        L.etd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != ETD_OK:
        raise EtdError(status, lib().etd_last_error().decode())


def problem_struct(p) -> etd_problem:
    """etd_problem from a workloads.Problem."""
    s = etd_problem()
    s.dim = p.dim
    for d in range(3):
        s.n[d] = p.n[d] if d < p.dim else 1
        s.lo[d] = p.lo[d]
        s.hi[d] = p.hi[d]
    s.ncomp = p.ncomp
    for c in range(p.ncomp):
        s.kappa[c] = p.kappa[c]
    s.q = p.q
    s.tau = p.tau
    s.rxn = RXN[p.reaction]
    for i, v in enumerate(p.params):
        s.rxn_param[i] = v
    s.pade = p.pade
    s.precision = PRECISION[p.precision]
    return s


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _field_spec(plan):
    """(element count, torch dtype) of a field of the plan's problem."""
    import torch
    pr = etd_plan_problem(plan)
    n = pr.ncomp
    for d in range(pr.dim):
        n *= pr.n[d]
    return n, (torch.float64 if pr.precision in (ETD_FP64, ETD_FP64_FP32, ETD_FP64_BF16X6) else torch.float32)


def _check_device(t, what):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor (got {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _check_field(plan, t, what="field", workspace=None):
    """Raise before any library call unless t is a contiguous device tensor of
    the plan's element type and field size (on the workspace's device)."""
    _check_device(t, what)
    n, dt = _field_spec(plan)
    if t.dtype != dt:
        raise ValueError(f"{what} has dtype {t.dtype}; the plan's precision needs {dt}")
    if t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} elements; the plan's field has {n}")
    if workspace is not None:
        _check_device(workspace, "workspace")
        if workspace.device != t.device:
            raise ValueError(f"{what} is on {t.device} but the workspace on {workspace.device}")


# --------------------------------------------------------------------------
# entry points (same names as include/etdds.h)
# --------------------------------------------------------------------------

def etd_plan_create(problem) -> ctypes.c_void_p:
    s = problem if isinstance(problem, etd_problem) else problem_struct(problem)
    h = ctypes.c_void_p()
    _check(lib().etd_plan_create(ctypes.byref(s), ctypes.byref(h)))
    return h


def etd_plan_workspace_bytes(plan) -> int:
    n = ctypes.c_size_t()
    _check(lib().etd_plan_workspace_bytes(plan, ctypes.byref(n)))
    return int(n.value)


def etd_plan_upload(plan, workspace, stream=None):
    _check(lib().etd_plan_upload(plan, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                 _stream(stream)))


def etd_advance(plan, u, t0: float, nsteps: int, workspace, stream=None):
    _check_field(plan, u, "field", workspace)
    _check(lib().etd_advance(plan, _ptr(u), float(t0), int(nsteps), _ptr(workspace), _stream(stream)))


def etd_compare(plan, a, b, workspace, stream=None, allow_nonfinite: bool = False):
    _check_field(plan, a, "a", workspace)
    _check_field(plan, b, "b", workspace)
    out = (ctypes.c_double * 4)()
    st = lib().etd_compare(plan, _ptr(a), _ptr(b), out, _ptr(workspace), _stream(stream))
    if not (allow_nonfinite and st == ETD_ENONFINITE):
        _check(st)
    return tuple(out)


def etd_compare_noalloc(plan, a, b, out, stream=None):
    """etd_compare without a workspace: the four results go to the device
    tensor `out` (4 float64), asynchronously on the stream."""
    import torch
    _check_field(plan, a, "a")
    _check_field(plan, b, "b")
    _check_device(out, "out")
    if out.dtype != torch.float64 or out.numel() < 4:
        raise ValueError("out must be a device float64 tensor of at least 4 elements")
    if a.device != b.device or out.device != a.device:
        raise ValueError("a, b and out must be on one device")
    _check(lib().etd_compare_noalloc(plan, _ptr(a), _ptr(b), _ptr(out), _stream(stream)))


def etd_plan_problem(plan) -> etd_problem:
    out = etd_problem()
    _check(lib().etd_plan_problem(plan, ctypes.byref(out)))
    return out


def etd_plan_table(plan, which: int, d: int, comp: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    _check(lib().etd_plan_table(plan, which, d, comp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                count))
    return out


def etd_timing_enable(plan, enable: bool = True):
    _check(lib().etd_timing_enable(plan, int(bool(enable))))


def etd_timing_read(plan):
    """(ms[3], counts[3]) per stage kind: 0 first outer, 1 middle outer, 2 x stage."""
    ms = (ctypes.c_double * 3)()
    cnt = (ctypes.c_longlong * 3)()
    _check(lib().etd_timing_read(plan, ms, cnt))
    return list(ms), list(cnt)


def etd_adjoint_workspace_bytes(plan, nsteps: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().etd_adjoint_workspace_bytes(plan, int(nsteps), ctypes.byref(n)))
    return int(n.value)


def etd_adjoint_workspace_bytes_segment(plan, nsteps: int, segment: int) -> int:
    """Adjoint workspace for checkpoint segments of `segment` steps (segment = nsteps: one forward pass)."""
    n = ctypes.c_size_t()
    _check(lib().etd_adjoint_workspace_bytes_segment(plan, int(nsteps), int(segment), ctypes.byref(n)))
    return int(n.value)


def etd_adjoint(plan, u0, t0: float, nsteps: int, ubar_final, ubar0, workspace, adjoint_workspace, ncomp: int,
                stream=None):
    """Returns [dL/dkappa_0, ..., dL/dkappa_{ncomp-1}, dL/dq]; writes dL/du0 into ubar0."""
    _check_field(plan, u0, "u0", workspace)
    _check_field(plan, ubar_final, "ubar_final", workspace)
    _check_field(plan, ubar0, "ubar0", workspace)
    _check_device(adjoint_workspace, "adjoint workspace")
    grad = (ctypes.c_double * (ncomp + 1))()
    nbytes = adjoint_workspace.numel() * adjoint_workspace.element_size()
    _check(lib().etd_adjoint(plan, _ptr(u0), float(t0), int(nsteps), _ptr(ubar_final), _ptr(ubar0), grad,
                             _ptr(workspace), _ptr(adjoint_workspace), nbytes, _stream(stream)))
    return list(grad)


def etd_plan_tiles(plan):
    """[(rows per wave, blocks)] per direction x, y, z ((0, 0) beyond dim)."""
    t = (ctypes.c_int * 6)()
    _check(lib().etd_plan_tiles(plan, t))
    return [(t[0], t[1]), (t[2], t[3]), (t[4], t[5])]


def etd_plan_set_tiles(plan, tiles):
    """tiles: up to three (rows per wave, blocks) pairs for x, y, z; (0, 0) = default."""
    flat = [0] * 6
    for d, (rb, cb) in enumerate(tiles):
        flat[2 * d], flat[2 * d + 1] = int(rb), int(cb)
    _check(lib().etd_plan_set_tiles(plan, (ctypes.c_int * 6)(*flat)))


SCHEDULE = {"auto": 0, "stages": 1, "resident": 2}


def etd_plan_set_schedule(plan, schedule):
    """schedule: "auto", "stages" or "resident" (or its ETD_SCHEDULE_* value)."""
    value = SCHEDULE[schedule] if isinstance(schedule, str) else int(schedule)
    _check(lib().etd_plan_set_schedule(plan, value))


def etd_plan_schedule(plan):
    """"stages" or "resident": the schedule etd_advance takes outside graph capture."""
    v = ctypes.c_int(-1)
    _check(lib().etd_plan_schedule(plan, ctypes.byref(v)))
    return {1: "stages", 2: "resident"}[v.value]


def etd_plan_autotune(plan, workspace, stream=None):
    _check(lib().etd_plan_autotune(plan, _ptr(workspace), _stream(stream)))


def etd_batch_create(problems) -> ctypes.c_void_p:
    arr = (etd_problem * len(problems))(*[p if isinstance(p, etd_problem) else problem_struct(p) for p in problems])
    h = ctypes.c_void_p()
    _check(lib().etd_batch_create(arr, len(problems), ctypes.byref(h)))
    return h


def etd_batch_workspace_bytes(batch) -> int:
    n = ctypes.c_size_t()
    _check(lib().etd_batch_workspace_bytes(batch, ctypes.byref(n)))
    return int(n.value)


def etd_batch_upload(batch, workspace, stream=None):
    _check(lib().etd_batch_upload(batch, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream(stream)))


def _ptr_array(fields):
    for i, f in enumerate(fields):
        _check_device(f, f"field {i}")
    return (ctypes.c_void_p * len(fields))(*[f.data_ptr() for f in fields])


def etd_batch_advance(batch, fields, t0: float, nsteps: int, workspace, stream=None):
    _check(lib().etd_batch_advance(batch, _ptr_array(fields), float(t0), int(nsteps), _ptr(workspace),
                                   _stream(stream)))


def etd_batch_autotune(batch, workspace, stream=None):
    _check(lib().etd_batch_autotune(batch, _ptr(workspace), _stream(stream)))


def etd_batch_tiles(batch, instance: int):
    t = (ctypes.c_int * 6)()
    _check(lib().etd_batch_tiles(batch, int(instance), t))
    return [(t[0], t[1]), (t[2], t[3]), (t[4], t[5])]


def etd_batch_groups(batch) -> int:
    n = ctypes.c_int()
    _check(lib().etd_batch_groups(batch, ctypes.byref(n)))
    return int(n.value)


def etd_batch_destroy(batch):
    _check(lib().etd_batch_destroy(batch))


def etd_graph_capture(plan, u, t0: float, nsteps: int, workspace, stream) -> ctypes.c_void_p:
    _check_field(plan, u, "field", workspace)
    h = ctypes.c_void_p()
    _check(lib().etd_graph_capture(plan, _ptr(u), float(t0), int(nsteps), _ptr(workspace), _stream(stream),
                                   ctypes.byref(h)))
    return h


def etd_batch_graph_capture(batch, fields, t0: float, nsteps: int, workspace, stream) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().etd_batch_graph_capture(batch, _ptr_array(fields), float(t0), int(nsteps), _ptr(workspace),
                                         _stream(stream), ctypes.byref(h)))
    return h


def etd_graph_launch(graph, stream=None):
    _check(lib().etd_graph_launch(graph, _stream(stream)))


def etd_graph_destroy(graph):
    _check(lib().etd_graph_destroy(graph))


def etd_plan_destroy(plan):
    _check(lib().etd_plan_destroy(plan))


def etd_status_string(status: int) -> str:
    return lib().etd_status_string(status).decode()


def etd_last_error() -> str:
    return lib().etd_last_error().decode()


# --------------------------------------------------------------------------
# convenience: plan + workspace owned together
# --------------------------------------------------------------------------

class Stepper:
    """A plan with its torch-allocated workspace on one device."""

    def __init__(self, problem, device="cuda:0", stream=None):
        import torch
        self.problem = problem
        self.device = torch.device(device)
        self.dtype = torch.float64 if problem.precision in FP64_STATE else torch.float32
        self.plan = etd_plan_create(problem)
        nbytes = etd_plan_workspace_bytes(self.plan)
        # over-allocate so the workspace can start on a 256-byte boundary
        self._raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._raw.data_ptr()) % 256
        self.workspace = self._raw[off:off + nbytes]
        self.stream = stream
        etd_plan_upload(self.plan, self.workspace, self.stream)

    def field(self, u0: np.ndarray):
        import torch
        return torch.as_tensor(np.ascontiguousarray(u0), dtype=self.dtype).reshape(self.problem.shape).to(
            self.device).contiguous()

    def advance(self, u, nsteps: int, t0: float = 0.0):
        etd_advance(self.plan, u, t0, nsteps, self.workspace, self.stream)
        return u

    def compare(self, a, b, allow_nonfinite=False):
        return etd_compare(self.plan, a, b, self.workspace, self.stream, allow_nonfinite)

    def adjoint_workspace(self, nsteps: int, segment: int = 0):
        """A 256-byte-aligned device buffer for adjoint(..., segment=segment)."""
        import torch
        nbytes = (etd_adjoint_workspace_bytes_segment(self.plan, nsteps, segment) if segment
                  else etd_adjoint_workspace_bytes(self.plan, nsteps))
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        return raw[off:off + nbytes]

    def adjoint(self, u0, ubar_final, nsteps: int, t0: float = 0.0, segment: int = 0, workspace=None):
        """(dL/du0, [dL/dkappa_c..., dL/dq]) for dL/dU_N = ubar_final.  segment:
        checkpoint segment length (0: the shortest, ceil(sqrt(nsteps)); nsteps:
        every step's stage fields kept, one forward pass); the adjoint takes the
        longest segment that fits `workspace` (allocated here when None)."""
        import torch
        aws = workspace if workspace is not None else self.adjoint_workspace(nsteps, segment)
        ubar0 = torch.empty(tuple(self.problem.shape), dtype=self.dtype, device=self.device)
        grad = etd_adjoint(self.plan, u0.contiguous(), t0, nsteps, ubar_final.contiguous(), ubar0, self.workspace,
                           aws, self.problem.ncomp, self.stream)
        return ubar0, grad

    def autotune(self):
        etd_plan_autotune(self.plan, self.workspace, self.stream)
        return self.tiles()

    def tiles(self):
        return etd_plan_tiles(self.plan)

    def set_tiles(self, tiles):
        etd_plan_set_tiles(self.plan, tiles)

    def set_schedule(self, schedule):
        etd_plan_set_schedule(self.plan, schedule)

    def schedule(self):
        return etd_plan_schedule(self.plan)

    def capture(self, u, nsteps: int, stream, t0: float = 0.0):
        """Graph of advance(u, nsteps, t0) captured from `stream` (not the null stream)."""
        return Graph(etd_graph_capture(self.plan, u, t0, nsteps, self.workspace, stream), (self, u))

    def close(self):
        if self.plan is not None:
            etd_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An executable HIP graph of captured stepper work (see etd_graph_capture)."""

    def __init__(self, handle, keepalive):
        self.handle = handle
        self._keep = keepalive   # objects whose memory the graph's kernels use

    def launch(self, stream=None):
        etd_graph_launch(self.handle, stream)

    def close(self):
        if self.handle is not None:
            etd_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent problems (same dim, ncomp, precision) advanced together
    by grouped persistent launches, with a torch-allocated workspace."""

    def __init__(self, problems, device="cuda:0", stream=None):
        import torch
        self.problems = list(problems)
        self.device = torch.device(device)
        self.dtype = torch.float64 if self.problems[0].precision in FP64_STATE else torch.float32
        self.batch = etd_batch_create(self.problems)
        nbytes = etd_batch_workspace_bytes(self.batch)
        self._raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._raw.data_ptr()) % 256
        self.workspace = self._raw[off:off + nbytes]
        self.stream = stream
        etd_batch_upload(self.batch, self.workspace, self.stream)

    def fields(self, u0s):
        import torch
        return [torch.as_tensor(np.ascontiguousarray(u), dtype=self.dtype).reshape(p.shape).to(self.device)
                .contiguous() for p, u in zip(self.problems, u0s)]

    def check_fields(self, fields):
        """Raise unless fields[i] is a contiguous device tensor of instance
        i's element type and size, on the batch's device."""
        if len(fields) != len(self.problems):
            raise ValueError(f"{len(fields)} fields for {len(self.problems)} instances")
        for i, (p, f) in enumerate(zip(self.problems, fields)):
            _check_device(f, f"field {i}")
            if f.dtype != self.dtype or f.numel() != int(np.prod(p.shape)) or f.device != self.workspace.device:
                raise ValueError(f"field {i}: {f.dtype} x {f.numel()} on {f.device}; instance {i} needs "
                                 f"{self.dtype} x {int(np.prod(p.shape))} on {self.workspace.device}")

    def advance(self, fields, nsteps: int, t0: float = 0.0):
        self.check_fields(fields)
        etd_batch_advance(self.batch, fields, t0, nsteps, self.workspace, self.stream)
        return fields

    def autotune(self):
        etd_batch_autotune(self.batch, self.workspace, self.stream)

    def tiles(self, instance: int):
        return etd_batch_tiles(self.batch, instance)

    def groups(self) -> int:
        return etd_batch_groups(self.batch)

    def capture(self, fields, nsteps: int, stream, t0: float = 0.0) -> Graph:
        self.check_fields(fields)
        h = etd_batch_graph_capture(self.batch, fields, t0, nsteps, self.workspace, stream)
        return Graph(h, (self, list(fields)))

    def close(self):
        if self.batch is not None:
            etd_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

# --------------------------------------------------------------------------
# autograd: U_N = advance(u0; kappa, q) with the hand-written adjoint
# --------------------------------------------------------------------------

def _autograd():
    import torch

    class EtdAdvance(torch.autograd.Function):
        """U_N after nsteps steps from u0; differentiable in u0, kappa and q
        through etd_adjoint (sqrt(N) checkpointing)."""

        @staticmethod
        def forward(ctx, u0, kappa, q, problem, nsteps, t0):
            p = problem.replace(kappa=tuple(float(k) for k in kappa.detach().cpu().reshape(-1)),
                                q=float(q.detach().cpu()))
            st = Stepper(p, device=u0.device)
            # the field in the plan's element type (an FP64 u0 for an FP32
            # problem is rounded once here; results come back as u0's dtype)
            u = u0.detach().to(st.dtype).clone().contiguous()
            ctx.save_for_backward(u.clone())
            st.advance(u, nsteps, t0)
            ctx.stepper, ctx.nsteps, ctx.t0 = st, nsteps, t0
            ctx.kshape, ctx.kdev, ctx.qdev = kappa.shape, kappa.device, q.device
            ctx.udtype = u0.dtype
            return u.to(u0.dtype)

        @staticmethod
        def backward(ctx, ubar):
            (u0,) = ctx.saved_tensors
            st = ctx.stepper
            ubar0, grad = st.adjoint(u0, ubar.to(st.dtype).contiguous(), ctx.nsteps, ctx.t0)
            ubar0 = ubar0.to(ctx.udtype)
            nc = st.problem.ncomp
            gk = torch.tensor(grad[:nc], dtype=torch.float64, device=ctx.kdev).reshape(ctx.kshape)
            gq = torch.tensor(grad[nc], dtype=torch.float64, device=ctx.qdev)
            return ubar0, gk, gq, None, None, None

    return EtdAdvance


def advance_autograd(u0, kappa, q, problem, nsteps: int, t0: float = 0.0):
    """Differentiable U_N (torch): gradients reach u0, kappa (one entry per
    component) and q through the hand-written adjoint."""
    return _autograd().apply(u0, kappa, q, problem, nsteps, t0)
