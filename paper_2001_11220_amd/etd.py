"""ctypes binding of ``libetdrdp.so`` (the C ABI in ``include/etd_rdp.h``).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the scheme runs in the library's kernels.
Importing this module loads the library and raises if it is missing, so no
caller can silently fall back to anything else.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libetdrdp.so")

ETD_OK = 0
ETD_ERR_ARG = -1
ETD_ERR_UNSUPPORTED = -2
ETD_ERR_WORKSPACE = -3
ETD_ERR_HIP = -4
ETD_ERR_INTERNAL = -5

BC = {"dirichlet": 0, "neumann": 1, "periodic": 2}
MODELS = {"linear": 0, "enzyme": 1, "brusselator": 2, "gray_scott": 3,
          "schnakenberg": 4, "cgl": 5, "cgl_z": 6, "nls_z": 7}
# parameter order of each model in etd_reaction_t.params
MODEL_PARAMS = {"enzyme": (), "brusselator": ("a", "b"), "gray_scott": ("F", "kappa"),
                "schnakenberg": ("a", "b", "gamma"), "cgl": ("beta",),
                "cgl_z": ("beta",), "nls_z": ("B", "C")}
SCHEMES = {"rdp": 0, "etd1": 1}
PRECISIONS = {"f64": 0, "f32": 1, "c128": 2}

MAX_DIM, MAX_SPECIES, MAX_PARAMS = 8, 2, 16


class Grid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("s", ctypes.c_int32),
                ("n", ctypes.c_int64 * MAX_DIM), ("h", ctypes.c_double * MAX_DIM)]


class Reaction(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("field", ctypes.c_int32),
                ("params", ctypes.c_double * MAX_PARAMS),
                ("shift", ctypes.c_double * MAX_SPECIES)]


class Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 2), ("h", ctypes.c_double * 2), ("bc", ctypes.c_int32 * 2),
                ("D", ctypes.c_double * MAX_SPECIES), ("params", ctypes.c_double * MAX_PARAMS),
                ("shift", ctypes.c_double * MAX_SPECIES)]


class Scheme(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("lines_per_wave", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class EtdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run `python -m paper_2001_11220_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "etd_rdp_init": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(I32), ctypes.POINTER(D), D,
                                        ctypes.POINTER(Scheme), ctypes.POINTER(Reaction), ctypes.POINTER(P)]),
        "etd_rdp_destroy": (ctypes.c_int, [P]),
        "etd_rdp_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "etd_rdp_workspace_layout": (ctypes.c_int, [P, I32, ctypes.POINTER(SZ), ctypes.POINTER(SZ),
                                                    ctypes.POINTER(SZ), ctypes.POINTER(I64)]),
        "etd_rdp_step": (ctypes.c_int, [P, P, P, SZ, I64, P]),
        "etd_rdp_step_f32": (ctypes.c_int, [P, P, P, SZ, I64, P]),
        "etd_rdp_step_z": (ctypes.c_int, [P, P, P, SZ, I64, P]),
        "etd_rdp_debug_passes": (ctypes.c_int, [P, P, P, SZ, I32, P]),
        "etd_rdp_run_pass": (ctypes.c_int, [P, P, P, SZ, I32, P]),
        "etd_rdp_run_pass_f32": (ctypes.c_int, [P, P, P, SZ, I32, P]),
        "etd_rdp_run_pass_z": (ctypes.c_int, [P, P, P, SZ, I32, P]),
        "etd_rdp_set_field": (ctypes.c_int, [P, P, SZ, P, P]),
        "etd_rdp_apply_solve": (ctypes.c_int, [P, P, P, SZ, I32, I32, I32, P]),
        "etd_rdp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "etd_rdp_last_hip_error": (ctypes.c_int, [P]),
        "etd_rdp_line_split": (ctypes.c_int, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "etd_rdp_pass_kernel": (ctypes.c_int, [P, I32, ctypes.c_char_p, SZ]),
        "etd_rdp_grad_size": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
        "etd_rdp_adjoint_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "etd_rdp_adjoint": (ctypes.c_int, [P, P, P, P, P, P, SZ, P]),
        "etd_rdp_batch_init": (ctypes.c_int, [I32, ctypes.POINTER(Instance), I32, I32, D,
                                              ctypes.POINTER(Scheme), ctypes.POINTER(P)]),
        "etd_rdp_batch_destroy": (ctypes.c_int, [P]),
        "etd_rdp_batch_offsets": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "etd_rdp_batch_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "etd_rdp_batch_step": (ctypes.c_int, [P, P, P, SZ, I64, I32, P]),
        "etd_rdp_batch_step_f32": (ctypes.c_int, [P, P, P, SZ, I64, I32, P]),
        "etd_rdp_batch_launches_per_step": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
        "etd_calib_stream": (ctypes.c_int, [I32, P, P, SZ, I32, P]),
        "etd_rdp_forget_workspace": (ctypes.c_int, [P]),
        "etd_rdp_batch_groups": (ctypes.c_int, [P, ctypes.POINTER(I32), P, P]),
        "etd_rdp_batch_get_plan": (ctypes.c_int, [P, P]),
        "etd_rdp_batch_set_plan": (ctypes.c_int, [P, P]),
        "etd_rdp_batch_form_allowed": (ctypes.c_int, [P, I32, I32, I32, ctypes.POINTER(I32)]),
        "etd_rdp_batch_tune": (ctypes.c_int, [P, P, P, SZ, I32, P, P]),
        "etd_rdp_batch_group_pass": (ctypes.c_int, [P, P, P, SZ, I32, I32, I32, P]),
        "etd_rdp_step_static": (ctypes.c_int, [P, P, I64, P]),
        "etd_rdp_set_slab": (ctypes.c_int, [P, I64]),
        "etd_rdp_set_graph": (ctypes.c_int, [P, I32]),
        "etd_rdp_record_graph": (ctypes.c_int, [P, P, P, SZ, I64]),
        "etd_rdp_get_slab": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "etd_rdp_batch_forget_workspace": (ctypes.c_int, [P]),
        "etd_rdp_keep_bytes": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "etd_rdp_step_keep": (ctypes.c_int, [P, P, P, P, SZ, P, SZ, P]),
        "etd_rdp_adjoint_kept": (ctypes.c_int, [P, P, P, SZ, P, P, P, P, SZ, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_string(status: int) -> str:
    return lib.etd_rdp_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != ETD_OK:
        raise EtdError(status, what)


def calib_stream(kind: str, src, dst, nbytes: int, blocks: int, stream=None):
    """One bandwidth-calibration sweep (etd_calib_stream) over torch device
    tensors: kind "copy" (src -> dst), "read" (src; dst a small sink),
    "write" (dst), "copy_nt" / "write_nt" (non-temporal stores) or
    "copy_ranges" (1024-thread blocks, one contiguous range each)."""
    import torch
    k = {"copy": 0, "read": 1, "write": 2, "copy_nt": 3, "write_nt": 4, "copy_ranges": 5}[kind]
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.etd_calib_stream(k, None if src is None else src.data_ptr(), dst.data_ptr(),
                                int(nbytes), int(blocks), ctypes.c_void_p(st.cuda_stream)),
           "etd_calib_stream")


def reaction_struct(model: str, params: dict, shift: Optional[Sequence[float]] = None,
                    s: int = 2) -> Reaction:
    rx = Reaction()
    rx.model = MODELS[model]
    if model == "linear":
        C = params["C"]
        flat = [float(v) for row in (C if hasattr(C[0], "__len__") else [C]) for v in row]
        for i, v in enumerate(flat):
            rx.params[i] = v
    else:
        for i, key in enumerate(MODEL_PARAMS[model]):
            rx.params[i] = float(params[key])
    sh = shift if shift is not None else params.get("shift")
    if sh is not None:
        for i, v in enumerate(sh):
            rx.shift[i] = float(v)
    return rx


class EtdRdp:
    """One ETD-RDP-IF problem on the GPU.

    ``shape`` is ``(n_1, ..., n_d)`` (axis 1 first); states are torch float64
    tensors of shape ``(s, n_d, ..., n_1)`` on a HIP device.  ``h`` entries of
    0 (or ``None``) select the unit-domain spacing of each boundary condition.
    ``lines_per_wave`` is "auto", 1, 2, 4 or 8 (ETD_LINES_* of the C ABI).
    ``precision`` "f32" makes the state and the carried arrays float32 (the
    reverse-mode step and the single solves stay "f64" only); "c128" is for
    one complex species (models "cgl_z", "nls_z", complex ``D``): states are
    complex128 tensors.
    """

    def __init__(self, shape, bcs, D, k, model, params, h=None, shift=None,
                 scheme="rdp", device=None, lines_per_wave="auto", precision="f64", field=False):
        d = len(shape)
        s = len(D)
        if not 1 <= d <= MAX_DIM:
            raise ValueError(f"{d}-D grid: the library takes up to {MAX_DIM} axes")
        g = Grid()
        g.d, g.s = d, s
        for i in range(d):
            g.n[i] = int(shape[i])
            g.h[i] = float(h[i]) if h is not None and h[i] is not None else 0.0
        bc_arr = (ctypes.c_int32 * MAX_DIM)(*[BC[b] if isinstance(b, str) else int(b) for b in bcs],
                                            *([0] * (MAX_DIM - d)))
        if precision == "c128":
            parts = [float(x) for v in D for x in (complex(v).real, complex(v).imag)]
            D_arr = (ctypes.c_double * (2 * MAX_SPECIES))(*parts, *([0.0] * (2 * MAX_SPECIES - 2 * s)))
        else:
            D_arr = (ctypes.c_double * MAX_SPECIES)(*[float(v) for v in D], *([0.0] * (MAX_SPECIES - s)))
        sch = Scheme()
        sch.scheme = SCHEMES[scheme]
        sch.lines_per_wave = 0 if lines_per_wave == "auto" else int(lines_per_wave)
        sch.precision = PRECISIONS[precision]
        self.precision = precision
        rx = reaction_struct(model, params, shift, s)
        rx.field = 1 if field else 0
        ctx = ctypes.c_void_p()
        _check(lib.etd_rdp_init(ctypes.byref(g), bc_arr, ctypes.cast(D_arr, ctypes.POINTER(ctypes.c_double)),
                                float(k), ctypes.byref(sch),
                                ctypes.byref(rx), ctypes.byref(ctx)), "etd_rdp_init")
        self._ctx = ctx
        self.shape, self.s, self.d = tuple(int(v) for v in shape), s, d
        self.D = tuple((complex(v) if precision == "c128" else float(v)) for v in D)
        self.model = model
        self._rx_params = tuple(float(rx.params[i]) for i in range(MAX_PARAMS))
        nb = ctypes.c_size_t()
        _check(lib.etd_rdp_workspace_bytes(ctx, ctypes.byref(nb)), "etd_rdp_workspace_bytes")
        self.ws_bytes = nb.value
        _check(lib.etd_rdp_adjoint_workspace_bytes(ctx, ctypes.byref(nb)),
               "etd_rdp_adjoint_workspace_bytes")
        self.adj_ws_bytes = nb.value
        gs = ctypes.c_int32()
        _check(lib.etd_rdp_grad_size(ctx, ctypes.byref(gs)), "etd_rdp_grad_size")
        self.grad_size = gs.value
        self._ws = None
        self._ws_cap = 0
        self._device = device

    def param_vector(self):
        """The values the gradient vector refers to: D, then the reaction
        parameters (params[] order)."""
        return list(self.D) + list(self._rx_params[: self.grad_size - self.s])

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            lib.etd_rdp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        self.close()

    # -- workspace ----------------------------------------------------------
    def workspace(self, nbytes=None):
        """Device workspace (a torch uint8 tensor owned by this object) of at
        least ``nbytes`` bytes (default: what a forward step needs).  Growing
        it replaces the buffer; the adjoint's workspace also serves forward
        steps."""
        import torch
        need = self.ws_bytes if nbytes is None else max(int(nbytes), self.ws_bytes)
        if self._ws is None or self._ws_cap < need:
            dev = self._device if self._device is not None else torch.device("cuda", torch.cuda.current_device())
            self._ws = None
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
            self._ws_cap = need
            # a new buffer, possibly at the old address: upload the tables again
            _check(lib.etd_rdp_forget_workspace(self._ctx), "etd_rdp_forget_workspace")
        return self._ws

    def _ws_ptr(self):
        ws = self.workspace()
        p = ws.data_ptr()
        return p + (-p) % 256

    def forget_workspace(self):
        """The workspace's contents were changed outside the library: the
        next call uploads the tables again (a reaction field must be set
        again)."""
        _check(lib.etd_rdp_forget_workspace(self._ctx), "etd_rdp_forget_workspace")

    def layout(self, npass=1):
        """(offsets of c1, c2, w in bytes, element strides of axes 1..d) of
        the carried triple pass ``npass`` writes."""
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        st = (ctypes.c_int64 * MAX_DIM)()
        _check(lib.etd_rdp_workspace_layout(self._ctx, int(npass), ctypes.byref(a), ctypes.byref(b),
                                            ctypes.byref(c), st), "etd_rdp_workspace_layout")
        return (a.value, b.value, c.value), tuple(int(st[i]) for i in range(self.d))

    def carried(self, npass=1):
        """Views (c1, c2, w) of the triple pass ``npass`` wrote, each with the
        state's logical shape (s, n_d, ..., n_1)."""
        import torch
        ws = self.workspace()
        base = self._ws_ptr() - ws.data_ptr()
        N = 1
        for v in self.shape:
            N *= v
        offs, strides = self.layout(npass)
        out = []
        for off in offs:
            flat = ws[base + off: base + off + 8 * N * self.s].view(torch.float64)
            out.append(flat.as_strided((self.s,) + self.shape[::-1], (N,) + strides[::-1]))
        return tuple(out)

    def pass_kernel(self, npass):
        """Name of the kernel pass ``npass`` launches (as profilers print it)."""
        buf = ctypes.create_string_buffer(64)
        _check(lib.etd_rdp_pass_kernel(self._ctx, int(npass), buf, 64), "etd_rdp_pass_kernel")
        return buf.value.decode()

    def line_split(self, axis):
        m, c = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.etd_rdp_line_split(self._ctx, axis, ctypes.byref(m), ctypes.byref(c)), "etd_rdp_line_split")
        return m.value, c.value

    # -- compute ------------------------------------------------------------
    def _state_ptr(self, u, nspecies, dtype=None):
        import torch
        want = (nspecies,) + self.shape[::-1]
        dt = dtype if dtype is not None else torch.float64
        if u.dtype != dt or not u.is_cuda or not u.is_contiguous() or tuple(u.shape) != want:
            raise ValueError(f"expected a contiguous {dt} device tensor of shape {want}")
        return u.data_ptr()

    def _elem_dtype(self):
        import torch
        return {"f32": torch.float32, "c128": torch.complex128}.get(self.precision, torch.float64)

    @staticmethod
    def _stream(stream):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(st.cuda_stream)

    def step(self, u, nsteps=1, stream=None):
        """Advance ``u`` in place by ``nsteps`` steps (asynchronous).  ``u`` is
        float64, float32 for a precision="f32" problem, complex128 for "c128"."""
        p = self._state_ptr(u, self.s, self._elem_dtype())
        fn, name = {"f32": (lib.etd_rdp_step_f32, "etd_rdp_step_f32"),
                    "c128": (lib.etd_rdp_step_z, "etd_rdp_step_z")}.get(
                        self.precision, (lib.etd_rdp_step, "etd_rdp_step"))
        _check(fn(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(self._ws_ptr()),
                  self.ws_bytes, int(nsteps), self._stream(stream)), name)
        return u

    @property
    def slab(self):
        """Planes of axis 3 per slab of passes 1-2 (0: whole passes)."""
        v = ctypes.c_int64()
        _check(lib.etd_rdp_get_slab(self._ctx, ctypes.byref(v)), "etd_rdp_get_slab")
        return v.value

    @slab.setter
    def slab(self, planes):
        _check(lib.etd_rdp_set_slab(self._ctx, int(planes)), "etd_rdp_set_slab")

    def use_graph(self, on=True):
        """Record step() calls into a HIP graph, replayed while (u, workspace,
        nsteps) repeat (etd_rdp_set_graph)."""
        _check(lib.etd_rdp_set_graph(self._ctx, 1 if on else 0), "etd_rdp_set_graph")

    def record_graph(self, u, nsteps):
        """Record (without running) the graph that step(u, nsteps) replays."""
        p = self._state_ptr(u, self.s, self._elem_dtype())
        _check(lib.etd_rdp_record_graph(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(self._ws_ptr()),
                                        self.ws_bytes, int(nsteps)), "etd_rdp_record_graph")

    def step_static(self, u, nsteps=1, stream=None):
        """``step`` with the library's own per-device workspace
        (etd_rdp_step_static): no allocation, FP64 problems whose workspace
        fits ETD_STATIC_SCRATCH_BYTES (64 MiB); calls that overlap on one
        device race."""
        p = self._state_ptr(u, self.s)
        _check(lib.etd_rdp_step_static(self._ctx, ctypes.c_void_p(p), int(nsteps),
                                       self._stream(stream)), "etd_rdp_step_static")
        return u

    def set_field(self, b, stream=None):
        """Store the per-cell reaction field ``b`` (a float64 device tensor
        shaped like one species, ``shape[::-1]``) of a ``field=True``
        problem in this object's workspace."""
        import torch
        want = self.shape[::-1]
        if b.dtype != torch.float64 or not b.is_cuda or not b.is_contiguous() or tuple(b.shape) != want:
            raise ValueError(f"expected a contiguous float64 device tensor of shape {want}")
        _check(lib.etd_rdp_set_field(self._ctx, ctypes.c_void_p(self._ws_ptr()), self.ws_bytes,
                                     ctypes.c_void_p(b.data_ptr()), self._stream(stream)), "etd_rdp_set_field")
        self._field_ref = b  # the copy is asynchronous on the stream

    def debug_passes(self, u, npasses, stream=None):
        p = self._state_ptr(u, self.s)
        _check(lib.etd_rdp_debug_passes(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(self._ws_ptr()),
                                        self.ws_bytes, int(npasses), self._stream(stream)),
               "etd_rdp_debug_passes")

    def run_pass(self, u, npass, stream=None):
        """Run pass ``npass`` (1..d) of a step alone (kernel timing)."""
        p = self._state_ptr(u, self.s, self._elem_dtype())
        fn, name = {"f32": (lib.etd_rdp_run_pass_f32, "etd_rdp_run_pass_f32"),
                    "c128": (lib.etd_rdp_run_pass_z, "etd_rdp_run_pass_z")}.get(
                        self.precision, (lib.etd_rdp_run_pass, "etd_rdp_run_pass"))
        _check(fn(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(self._ws_ptr()),
                  self.ws_bytes, int(npass), self._stream(stream)), name)

    def adjoint(self, u_n, lam, lam_out=None, grad=None, stream=None, kept=None):
        """One reverse step: returns (dL/dU_n, grad) for lam = dL/dU_{n+1}.
        ``grad`` (float64 device tensor of ``grad_size``) is accumulated into;
        a zero one is made if it is None.  ``lam_out`` may be ``lam``.
        ``kept``: the arrays ``step_keep`` left for the step from ``u_n``
        (the reverse step then skips recomputing them)."""
        import torch
        pu = self._state_ptr(u_n, self.s)
        pl = self._state_ptr(lam, self.s)
        if lam_out is None:
            lam_out = torch.empty_like(lam)
        po = self._state_ptr(lam_out, self.s)
        if grad is None:
            grad = torch.zeros(self.grad_size, dtype=torch.float64, device=lam.device)
        if grad.dtype != torch.float64 or not grad.is_cuda or not grad.is_contiguous() or grad.numel() != self.grad_size:
            raise ValueError(f"grad must be a contiguous float64 device tensor of {self.grad_size}")
        self.workspace(self.adj_ws_bytes)
        if kept is not None:
            _check(lib.etd_rdp_adjoint_kept(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(self._keep_ptr(kept)),
                                            kept.numel() * 8, ctypes.c_void_p(pl), ctypes.c_void_p(po),
                                            ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(self._ws_ptr()),
                                            self._ws_cap, self._stream(stream)), "etd_rdp_adjoint_kept")
            return lam_out, grad
        _check(lib.etd_rdp_adjoint(self._ctx, ctypes.c_void_p(pu), ctypes.c_void_p(pl), ctypes.c_void_p(po),
                                   ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(self._ws_ptr()),
                                   self._ws_cap, self._stream(stream)), "etd_rdp_adjoint")
        return lam_out, grad

    @property
    def keep_bytes(self):
        """Bytes of one step's kept carried arrays (etd_rdp_keep_bytes)."""
        nb = ctypes.c_size_t()
        _check(lib.etd_rdp_keep_bytes(self._ctx, ctypes.byref(nb)), "etd_rdp_keep_bytes")
        return nb.value

    def new_keep(self, count=1):
        """A float64 device tensor holding ``count`` steps' kept arrays
        (``keep[i]`` for step i)."""
        import torch
        n = self.keep_bytes // 8
        dev = self._device if self._device is not None else torch.device("cuda", torch.cuda.current_device())
        return torch.empty((count, n), dtype=torch.float64, device=dev)

    def _keep_ptr(self, keep):
        import torch
        if keep.dtype != torch.float64 or not keep.is_cuda or not keep.is_contiguous() or \
                keep.numel() * 8 < self.keep_bytes or keep.data_ptr() % 256 != 0:
            raise ValueError("keep must be a contiguous, 256-byte aligned float64 device tensor "
                             f"of at least {self.keep_bytes} bytes (see new_keep)")
        return keep.data_ptr()

    def step_keep(self, u, keep, out=None, stream=None):
        """One step of ``u`` into ``out`` (``u`` itself when None, in place),
        its carried arrays left in ``keep`` (one row of ``new_keep()``) for
        ``adjoint(..., kept=keep)``.  Returns the stepped state."""
        p = self._state_ptr(u, self.s)
        if out is None:
            out = u
        po = self._state_ptr(out, self.s)
        _check(lib.etd_rdp_step_keep(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(po),
                                     ctypes.c_void_p(self._ws_ptr()), self._ws_cap,
                                     ctypes.c_void_p(self._keep_ptr(keep)), keep.numel() * 8,
                                     self._stream(stream)), "etd_rdp_step_keep")
        return out

    def apply_solve(self, x, axis, sigma, gamma, stream=None):
        p = self._state_ptr(x, 1)
        _check(lib.etd_rdp_apply_solve(self._ctx, ctypes.c_void_p(p), ctypes.c_void_p(self._ws_ptr()),
                                       self.ws_bytes, int(axis), int(sigma), int(gamma),
                                       self._stream(stream)), "etd_rdp_apply_solve")
        return x


class EtdRdpBatch:
    """An ensemble of independent 2-D problems advanced together.

    ``instances``: sequence of dicts with keys ``shape`` (n_1, n_2), ``bcs``,
    ``D`` and ``params`` (and optionally ``h``, ``shift``).  The packed state
    is one device tensor of ``offsets[-1]`` elements (float64, or float32
    with ``precision="f32"``); instance i is
    ``u[offsets[i]: offsets[i] + s*n_1*n_2]`` viewed as ``(s, n_2, n_1)``.
    """

    def __init__(self, instances, s, model, k, scheme="rdp", device=None, precision="f64"):
        if precision not in ("f64", "f32"):
            raise ValueError(f"ensembles run in f64 or f32, not {precision!r}")
        n = len(instances)
        arr = (Instance * n)()
        for i, ins in enumerate(instances):
            a = arr[i]
            for q in range(2):
                a.n[q] = int(ins["shape"][q])
                h = ins.get("h")
                a.h[q] = float(h[q]) if h is not None and h[q] else 0.0
                b = ins["bcs"][q]
                a.bc[q] = BC[b] if isinstance(b, str) else int(b)
            for q, v in enumerate(ins["D"]):
                a.D[q] = float(v)
            rx = reaction_struct(model, ins["params"], ins.get("shift"), s)
            for q in range(MAX_PARAMS):
                a.params[q] = rx.params[q]
            for q in range(MAX_SPECIES):
                a.shift[q] = rx.shift[q]
        sch = Scheme()
        sch.scheme = SCHEMES[scheme]
        sch.precision = PRECISIONS[precision]
        ctx = ctypes.c_void_p()
        _check(lib.etd_rdp_batch_init(n, arr, int(s), MODELS[model], float(k), ctypes.byref(sch),
                                      ctypes.byref(ctx)), "etd_rdp_batch_init")
        self._ctx = ctx
        self.n, self.s = n, int(s)
        self.precision = precision
        self.model, self.scheme = model, scheme
        self.shapes = [tuple(int(v) for v in ins["shape"]) for ins in instances]
        offs = (ctypes.c_int64 * (n + 1))()
        _check(lib.etd_rdp_batch_offsets(ctx, offs), "etd_rdp_batch_offsets")
        self.offsets = [int(v) for v in offs]
        nb = ctypes.c_size_t()
        _check(lib.etd_rdp_batch_workspace_bytes(ctx, ctypes.byref(nb)), "etd_rdp_batch_workspace_bytes")
        self.ws_bytes = nb.value
        lp = ctypes.c_int32()
        _check(lib.etd_rdp_batch_launches_per_step(ctx, ctypes.byref(lp)), "etd_rdp_batch_launches_per_step")
        self.launches_per_step = lp.value
        self._ws = None
        self._device = device

    def close(self):
        if getattr(self, "_ctx", None):
            lib.etd_rdp_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        self.close()

    def workspace(self):
        import torch
        if self._ws is None:
            dev = self._device if self._device is not None else torch.device("cuda", torch.cuda.current_device())
            self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
            _check(lib.etd_rdp_batch_forget_workspace(self._ctx), "etd_rdp_batch_forget_workspace")
        return self._ws

    def _ws_ptr(self):
        ws = self.workspace()
        p = ws.data_ptr()
        return p + (-p) % 256

    FORMS = ("unsplit", "streamed", "two_line")

    def groups(self):
        """[(n1, n2, instances)] of the ensemble's groups (instances of one
        grid shape, one launch per pass each)."""
        ng = ctypes.c_int32()
        _check(lib.etd_rdp_batch_groups(self._ctx, ctypes.byref(ng), None, None), "etd_rdp_batch_groups")
        shapes = (ctypes.c_int64 * (2 * ng.value))()
        counts = (ctypes.c_int32 * ng.value)()
        _check(lib.etd_rdp_batch_groups(self._ctx, ctypes.byref(ng), shapes, counts), "etd_rdp_batch_groups")
        return [(int(shapes[2 * g]), int(shapes[2 * g + 1]), int(counts[g])) for g in range(ng.value)]

    @property
    def plan(self):
        """Kernel form of every (group, pass): plan[2 g + p] in ETD_FORM_*."""
        n = 2 * len(self.groups())
        arr = (ctypes.c_int32 * n)()
        _check(lib.etd_rdp_batch_get_plan(self._ctx, arr), "etd_rdp_batch_get_plan")
        return [int(v) for v in arr]

    @plan.setter
    def plan(self, plan):
        arr = (ctypes.c_int32 * len(plan))(*[int(v) for v in plan])
        if len(plan) != 2 * len(self.groups()):
            raise ValueError("a plan has two entries per group")
        _check(lib.etd_rdp_batch_set_plan(self._ctx, arr), "etd_rdp_batch_set_plan")

    def form_allowed(self, group, npass, form):
        v = ctypes.c_int32()
        _check(lib.etd_rdp_batch_form_allowed(self._ctx, int(group), int(npass), int(form), ctypes.byref(v)),
               "etd_rdp_batch_form_allowed")
        return bool(v.value)

    def tune(self, u, reps=3, stream=None):
        """Run the library's autotuner on the packed state ``u`` (advanced by
        one step): every allowed form of every (group, pass) is timed and the
        fastest kept in the plan.  Returns times[group][pass][form] in ms per
        launch (None where a form is not allowed)."""
        import torch
        if u.dtype != self.dtype or not u.is_cuda or not u.is_contiguous() or u.numel() != self.offsets[-1]:
            raise ValueError(f"expected the packed contiguous {self.dtype} device state")
        ng = len(self.groups())
        times = (ctypes.c_double * (6 * ng))()
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib.etd_rdp_batch_tune(self._ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(self._ws_ptr()),
                                      self.ws_bytes, int(reps), ctypes.c_void_p(st.cuda_stream), times),
               "etd_rdp_batch_tune")
        return [[[None if times[(2 * g + p) * 3 + f] < 0 else float(times[(2 * g + p) * 3 + f])
                  for f in range(3)] for p in range(2)] for g in range(ng)]

    def group_pass(self, u, group, npass, form=-1, stream=None):
        """Launch one pass of one group alone (pass 0 reads u and writes the
        carried arrays, pass 1 reads them and writes u)."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib.etd_rdp_batch_group_pass(self._ctx, ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(self._ws_ptr()), self.ws_bytes, int(group),
                                            int(npass), int(form), ctypes.c_void_p(st.cuda_stream)),
               "etd_rdp_batch_group_pass")

    def forget_workspace(self):
        """The workspace's contents were changed outside the library: the
        next step uploads the tables again and records a new graph."""
        _check(lib.etd_rdp_batch_forget_workspace(self._ctx), "etd_rdp_batch_forget_workspace")

    def pack(self, states):
        """Pack per-instance numpy/torch states (s, n_2, n_1) into one
        torch tensor of the ensemble's dtype (on the workspace's device)."""
        import torch
        ws = self.workspace()
        u = torch.zeros(self.offsets[-1], dtype=self.dtype, device=ws.device)
        for i, st in enumerate(states):
            t = torch.as_tensor(st).to(self.dtype).reshape(-1)
            u[self.offsets[i]: self.offsets[i] + t.numel()] = t.to(ws.device)
        return u

    def view(self, u, i):
        n1, n2 = self.shapes[i]
        return u[self.offsets[i]: self.offsets[i] + self.s * n1 * n2].view(self.s, n2, n1)

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.precision == "f32" else torch.float64

    def step(self, u, nsteps=1, use_graph=True, stream=None):
        import torch
        if u.dtype != self.dtype or not u.is_cuda or not u.is_contiguous() or u.numel() != self.offsets[-1]:
            raise ValueError(f"expected the packed contiguous {self.dtype} device state")
        st = stream if stream is not None else torch.cuda.current_stream()
        name = "etd_rdp_batch_step_f32" if self.precision == "f32" else "etd_rdp_batch_step"
        _check(getattr(lib, name)(self._ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(self._ws_ptr()),
                                  self.ws_bytes, int(nsteps), 1 if use_graph else 0,
                                  ctypes.c_void_p(st.cuda_stream)), name)
        return u
