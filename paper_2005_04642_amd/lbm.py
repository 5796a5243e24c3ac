"""Thin Python binding of the C ABI in include/chromo_lbm.h.

The functions keep the C names (``lbm_init``, ``lbm_step``, ``lbm_fields``,
...) and only marshal arguments: every step of the scheme runs in the HIP
library.  PyTorch provides device memory and the current stream.  There is no
CPU fallback: if the library is missing or no GPU is present the calls raise.

``Simulation`` bundles the buffers one lattice needs (two population buffers,
the workspace, the initial colour index and the optional force field).
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libchromo_lbm.so")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENOTIMPL, LBM_ENONFINITE = 0, -1, -2, -3, -4
LBM_STORAGE_F64, LBM_STORAGE_F32, LBM_STORAGE_F16_OFS, LBM_STORAGE_BF16_OFS = 0, 1, 2, 3
STORAGE = {"f64": LBM_STORAGE_F64, "f32": LBM_STORAGE_F32, "f16": LBM_STORAGE_F16_OFS, "bf16": LBM_STORAGE_BF16_OFS}
WORDS_PER_SITE = {"f64": 18, "f32": 18, "f16": 10, "bf16": 10}
LBM_FLAG_STREAM_ONLY, LBM_FLAG_FIXED_K, LBM_FLAG_NO_RECOLOR, LBM_FLAG_MASK_PASSES = 1, 2, 4, 8

# every symbol the header declares
EXPORTED = ("lbm_validate_params", "lbm_pops_elems", "lbm_pops_bytes", "lbm_workspace_bytes", "lbm_init",
            "lbm_step", "lbm_step_static", "lbm_step_into", "lbm_fields", "lbm_masses_host",
            "lbm_adjoint_workspace_bytes", "lbm_adjoint_step", "lbm_adjoint_steps",
            "lbm_rhoN_adjoint", "lbm_init_adjoint", "lbm_solid_workspace_bytes", "lbm_set_solid",
            "lbm_current_pops", "lbm_set_pops", "lbm_step_count", "lbm_set_cu_budget", "lbm_partition_stream",
            "lbm_destroy", "lbm_last_error", "lbm_batch_pops_bytes", "lbm_batch_offsets", "lbm_batch_workspace_bytes",
            "lbm_batch_init", "lbm_batch_step", "lbm_batch_autotune", "lbm_batch_set_force", "lbm_batch_set_solid",
            "lbm_batch_plan_info",
            "lbm_batch_fields",
            "lbm_batch_masses_host", "lbm_batch_current_pops", "lbm_batch_step_count", "lbm_batch_destroy")


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm status %d: %s" % (code, msg))
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls_y", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("stencil", ctypes.c_int32 * 4), ("ghost_eq", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("rho0_R", ctypes.c_double), ("rho0_B", ctypes.c_double),
                ("alpha_R", ctypes.c_double), ("alpha_B", ctypes.c_double),
                ("nu_R", ctypes.c_double), ("nu_B", ctypes.c_double),
                ("sigma", ctypes.c_double), ("beta", ctypes.c_double),
                ("lambda6", ctypes.c_double), ("lambda7", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("K_fixed", ctypes.c_double), ("eps_n", ctypes.c_double)]


_lib = None


def load_library(path=None):
    """Load libchromo_lbm.so (built in-tree by ``build_lib.build()``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("HIP library %s is missing: run paper_2005_04642_amd.build_lib.build()" % p)
    lib = ctypes.CDLL(p)
    vp, i32, sz, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(lbm_params)
    lib.lbm_validate_params.argtypes = [P]
    lib.lbm_validate_params.restype = ctypes.c_int
    lib.lbm_pops_elems.argtypes = [P]
    lib.lbm_pops_elems.restype = sz
    lib.lbm_pops_bytes.argtypes = [P]
    lib.lbm_pops_bytes.restype = sz
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = sz
    lib.lbm_init.argtypes = [P, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    lib.lbm_init.restype = ctypes.c_int
    lib.lbm_step.argtypes = [vp, i32, vp, vp]
    lib.lbm_step.restype = ctypes.c_int
    lib.lbm_step_static.argtypes = [vp, i32, vp, vp]
    lib.lbm_step_static.restype = ctypes.c_int
    lib.lbm_fields.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.lbm_fields.restype = ctypes.c_int
    lib.lbm_masses_host.argtypes = [vp, dp, vp]
    lib.lbm_masses_host.restype = ctypes.c_int
    lib.lbm_adjoint_workspace_bytes.argtypes = [P]
    lib.lbm_adjoint_workspace_bytes.restype = sz
    lib.lbm_adjoint_step.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp, vp]
    lib.lbm_adjoint_step.restype = ctypes.c_int
    lib.lbm_adjoint_steps.argtypes = [vp, i32, ctypes.POINTER(vp), vp, vp, vp, sz, vp, vp, vp]
    lib.lbm_adjoint_steps.restype = ctypes.c_int
    lib.lbm_step_into.argtypes = [vp, vp, i32, ctypes.POINTER(vp), vp]
    lib.lbm_step_into.restype = ctypes.c_int
    lib.lbm_rhoN_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_rhoN_adjoint.restype = ctypes.c_int
    lib.lbm_init_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_init_adjoint.restype = ctypes.c_int
    lib.lbm_solid_workspace_bytes.argtypes = [P]
    lib.lbm_solid_workspace_bytes.restype = sz
    lib.lbm_set_solid.argtypes = [vp, vp, vp, sz, vp]
    lib.lbm_set_solid.restype = ctypes.c_int
    lib.lbm_current_pops.argtypes = [vp]
    lib.lbm_current_pops.restype = ctypes.c_int
    lib.lbm_set_pops.argtypes = [vp, vp, vp]
    lib.lbm_set_pops.restype = ctypes.c_int
    lib.lbm_step_count.argtypes = [vp]
    lib.lbm_step_count.restype = ctypes.c_int64
    lib.lbm_set_cu_budget.argtypes = [vp, i32, i32]
    lib.lbm_set_cu_budget.restype = ctypes.c_int
    lib.lbm_partition_stream.argtypes = [i32, i32, ctypes.POINTER(vp)]
    lib.lbm_partition_stream.restype = ctypes.c_int
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.lbm_batch_pops_bytes.argtypes = [P, ctypes.c_int]
    lib.lbm_batch_pops_bytes.restype = sz
    lib.lbm_batch_offsets.argtypes = [P, ctypes.c_int, ctypes.POINTER(sz)]
    lib.lbm_batch_offsets.restype = ctypes.c_int
    lib.lbm_batch_workspace_bytes.argtypes = [P, ctypes.c_int]
    lib.lbm_batch_workspace_bytes.restype = sz
    lib.lbm_batch_init.argtypes = [P, ctypes.c_int, ctypes.POINTER(vp), vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
    lib.lbm_batch_init.restype = ctypes.c_int
    lib.lbm_batch_step.argtypes = [vp, i32, vp]
    lib.lbm_batch_step.restype = ctypes.c_int
    lib.lbm_batch_autotune.argtypes = [vp, vp, sz, i32, vp, i32p]
    lib.lbm_batch_autotune.restype = ctypes.c_int
    lib.lbm_batch_set_force.argtypes = [vp, i32, vp, vp]
    lib.lbm_batch_set_force.restype = ctypes.c_int
    lib.lbm_batch_set_solid.argtypes = [vp, i32, vp, vp, sz, vp]
    lib.lbm_batch_set_solid.restype = ctypes.c_int
    lib.lbm_batch_plan_info.argtypes = [vp, i32p]
    lib.lbm_batch_plan_info.restype = ctypes.c_int
    lib.lbm_batch_fields.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.lbm_batch_fields.restype = ctypes.c_int
    lib.lbm_batch_masses_host.argtypes = [vp, i32, dp, vp]
    lib.lbm_batch_masses_host.restype = ctypes.c_int
    lib.lbm_batch_current_pops.argtypes = [vp]
    lib.lbm_batch_current_pops.restype = ctypes.c_int
    lib.lbm_batch_step_count.argtypes = [vp]
    lib.lbm_batch_step_count.restype = ctypes.c_int64
    lib.lbm_batch_destroy.argtypes = [vp]
    lib.lbm_batch_destroy.restype = None
    if path is None:
        _lib = lib
    return lib


def _check(lib, code):
    if code != LBM_OK:
        raise LbmError(code, lib.lbm_last_error().decode())
    return code


def make_params(nx, ny, storage="f32", **kw):
    """lbm_params from keyword parameters (the dictionaries of ``workloads``)."""
    p = lbm_params()
    p.nx, p.ny = nx, ny
    p.walls_y = 1 if kw.get("walls", False) else 0
    p.storage = STORAGE[storage]
    st = kw.get("stencil", (3, 3, 3, 3))
    for k in range(4):
        p.stencil[k] = int(st[k])
    p.ghost_eq = int(kw.get("ghost_eq", 0))
    flags = int(kw.get("flags", 0))
    if kw.get("fixed_K") is not None:
        flags |= LBM_FLAG_FIXED_K
        p.K_fixed = float(kw["fixed_K"])
    if not kw.get("recolor", True):
        flags |= LBM_FLAG_NO_RECOLOR
    p.flags = flags
    for name in ("rho0_R", "rho0_B", "alpha_R", "alpha_B", "nu_R", "nu_B", "sigma", "beta",
                 "lambda6", "lambda7", "gx", "gy"):
        setattr(p, name, float(kw[name]) if name in kw else 0.0)
    p.eps_n = float(kw.get("eps_n", 1e-6))
    return p


# ---------------------------------------------------------------------------
# C-name wrappers (argument marshalling only)
# ---------------------------------------------------------------------------

def lbm_validate_params(p):
    lib = load_library()
    return lib.lbm_validate_params(ctypes.byref(p)), lib.lbm_last_error().decode()


def lbm_pops_elems(p):
    return load_library().lbm_pops_elems(ctypes.byref(p))


def lbm_pops_bytes(p):
    return load_library().lbm_pops_bytes(ctypes.byref(p))


def lbm_workspace_bytes(p):
    return load_library().lbm_workspace_bytes(ctypes.byref(p))


def lbm_init(p, rhoN0_ptr, force_ptr, pops_a_ptr, pops_b_ptr, ws_ptr, ws_bytes, stream):
    lib = load_library()
    h = ctypes.c_void_p()
    _check(lib, lib.lbm_init(ctypes.byref(p), rhoN0_ptr, force_ptr, pops_a_ptr, pops_b_ptr, ws_ptr,
                             ws_bytes, stream, ctypes.byref(h)))
    return h


def lbm_step(h, nsteps, mass_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_step(h, nsteps, mass_ptr, stream))


def lbm_step_static(h, nsteps, mass_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_step_static(h, nsteps, mass_ptr, stream))


def lbm_fields(h, rho_ptr, ux_ptr, uy_ptr, rhoN_ptr, mass_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_fields(h, rho_ptr, ux_ptr, uy_ptr, rhoN_ptr, mass_ptr, stream))


def lbm_masses_host(h, stream):
    lib = load_library()
    out = (ctypes.c_double * 2)()
    _check(lib, lib.lbm_masses_host(h, out, stream))
    return out[0], out[1]


def lbm_adjoint_workspace_bytes(p):
    return load_library().lbm_adjoint_workspace_bytes(ctypes.byref(p))


def lbm_adjoint_step(h, pops_t_ptr, adj_next_ptr, adj_out_ptr, ws_ptr, ws_bytes, dsigma_ptr, dforce_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_adjoint_step(h, pops_t_ptr, adj_next_ptr, adj_out_ptr, ws_ptr, ws_bytes, dsigma_ptr,
                                            dforce_ptr, stream))


def lbm_adjoint_steps(h, state_ptrs, adj_a_ptr, adj_b_ptr, ws_ptr, ws_bytes, dsigma_ptr, dforce_ptr, stream):
    """len(state_ptrs) adjoint steps backwards through the states (device
    pointers, oldest first); the result is in adj_a for an even count, else
    adj_b."""
    lib = load_library()
    n = len(state_ptrs)
    arr = (ctypes.c_void_p * max(n, 1))(*state_ptrs)
    return _check(lib, lib.lbm_adjoint_steps(h, n, arr, adj_a_ptr, adj_b_ptr, ws_ptr, ws_bytes, dsigma_ptr,
                                             dforce_ptr, stream))


def lbm_step_into(h, from_ptr, state_ptrs, stream):
    """len(state_ptrs) steps from the state at from_ptr, the state after
    step j written to state_ptrs[j]."""
    lib = load_library()
    n = len(state_ptrs)
    arr = (ctypes.c_void_p * max(n, 1))(*state_ptrs)
    return _check(lib, lib.lbm_step_into(h, from_ptr, n, arr, stream))


def lbm_rhoN_adjoint(h, pops_ptr, dL_drhoN_ptr, adj_out_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_rhoN_adjoint(h, pops_ptr, dL_drhoN_ptr, adj_out_ptr, stream))


def lbm_init_adjoint(h, rhoN0_ptr, adj0_ptr, dL_drhoN0_ptr, stream):
    lib = load_library()
    return _check(lib, lib.lbm_init_adjoint(h, rhoN0_ptr, adj0_ptr, dL_drhoN0_ptr, stream))


def lbm_solid_workspace_bytes(p):
    return load_library().lbm_solid_workspace_bytes(ctypes.byref(p))


def lbm_set_solid(h, solid_ptr, ws_ptr, ws_bytes, stream):
    lib = load_library()
    return _check(lib, lib.lbm_set_solid(h, solid_ptr, ws_ptr, ws_bytes, stream))


def lbm_current_pops(h):
    return load_library().lbm_current_pops(h)


def lbm_set_pops(h, live_ptr, next_ptr):
    lib = load_library()
    return _check(lib, lib.lbm_set_pops(h, live_ptr, next_ptr))


def lbm_step_count(h):
    return load_library().lbm_step_count(h)


def lbm_set_cu_budget(h, ncu_step, ncu_adjoint):
    lib = load_library()
    return _check(lib, lib.lbm_set_cu_budget(h, int(ncu_step), int(ncu_adjoint)))


def lbm_partition_stream(cu_first, cu_count):
    """A new HIP stream (as an int handle) confined to CUs [cu_first,
    cu_first + cu_count) of the current device; the caller owns it."""
    lib = load_library()
    out = ctypes.c_void_p()
    _check(lib, lib.lbm_partition_stream(int(cu_first), int(cu_count), ctypes.byref(out)))
    return out.value


def lbm_destroy(h):
    load_library().lbm_destroy(h)


def lbm_last_error():
    return load_library().lbm_last_error().decode()


# ---------------------------------------------------------------------------
# convenience: one lattice with torch-owned device buffers
# ---------------------------------------------------------------------------

class Simulation:
    """Buffers and handle of one lattice.

    params: dict of physical parameters (see ``workloads.base_params``);
    rhoN0: [ny, nx] initial colour index (numpy or torch); storage 'f64',
    'f32', or the 16-bit offset formats 'f16' / 'bf16' (FP32 arithmetic);
    force: optional [2, ny, nx] per-site body force density; solid: optional
    [ny, nx] mask of solid sites (lbm_set_solid; F64/F32 storage, no walls).
    Fields, rhoN0 and force use the arithmetic type (float64 for 'f64', else
    float32).
    """

    def __init__(self, nx, ny, params, rhoN0, storage="f32", force=None, device="cuda:0", flags=0, solid=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the chromodynamic LBM step runs only on the HIP device")
        self.torch = torch
        self.nx, self.ny = nx, ny
        self.device = torch.device(device)
        kw = dict(params)
        kw["flags"] = kw.get("flags", 0) | flags
        self.params = make_params(nx, ny, storage, **kw)
        self.storage = storage
        self.dtype = torch.float64 if storage == "f64" else torch.float32
        self.word_dtype = {"f64": torch.float64, "f32": torch.float32}.get(storage, torch.int32)
        code, msg = lbm_validate_params(self.params)
        if code != LBM_OK:
            raise LbmError(code, msg)
        n = lbm_pops_elems(self.params)
        self.pops = [torch.empty(n, dtype=self.word_dtype, device=self.device) for _ in range(2)]
        wsb = lbm_workspace_bytes(self.params)
        self.ws = torch.zeros(wsb, dtype=torch.uint8, device=self.device)
        def dev(a):
            t = a if torch.is_tensor(a) else torch.as_tensor(np.asarray(a))
            return t.to(device=self.device, dtype=self.dtype).contiguous()

        self.rhoN0 = dev(rhoN0)
        self.force = None if force is None else dev(force)
        self.mass = torch.zeros(2, dtype=torch.float64, device=self.device)
        self.h = lbm_init(self.params, self.rhoN0.data_ptr(),
                          None if self.force is None else self.force.data_ptr(),
                          self.pops[0].data_ptr(), self.pops[1].data_ptr(), self.ws.data_ptr(), wsb,
                          self.stream())
        self.solid = None
        if solid is not None:
            self.set_solid(solid)

    def set_solid(self, solid):
        """Give the lattice a mask of solid sites ([ny, nx], nonzero = solid),
        keeping the pre-collision populations of the fluid sites."""
        t = self.torch
        m = solid if t.is_tensor(solid) else t.as_tensor(np.asarray(solid))
        m = (m != 0).to(device=self.device, dtype=t.uint8).contiguous()
        if tuple(m.shape) != (self.ny, self.nx):
            raise ValueError("solid mask must have shape (ny, nx)")
        n = lbm_solid_workspace_bytes(self.params)
        if n == 0:
            raise LbmError(LBM_ENOTIMPL, "no solid-site mask for these parameters (needs F64/F32 storage, no walls)")
        ws = t.empty(n, dtype=t.uint8, device=self.device)
        lbm_set_solid(self.h, m.data_ptr(), ws.data_ptr(), n, self.stream())
        self.solid, self._solid_ws = m, ws   # both must outlive the handle's use of them

    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def step(self, n=1, with_mass=False):
        lbm_step(self.h, int(n), self.mass.data_ptr() if with_mass else None, self.stream())
        return self

    def set_cu_budget(self, step=0, adjoint=0):
        """Plan the forward step's tiles for `step` CUs and the adjoint's first
        pass for `adjoint` CUs (0: the whole device), for work run on streams
        confined to that many CUs (lbm_partition_stream)."""
        lbm_set_cu_budget(self.h, step, adjoint)
        return self

    def fields(self):
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=self.dtype, device=self.device)
               for k in ("rho", "ux", "uy", "rhoN")}
        lbm_fields(self.h, out["rho"].data_ptr(), out["ux"].data_ptr(), out["uy"].data_ptr(),
                   out["rhoN"].data_ptr(), None, self.stream())
        return out

    def masses(self):
        return lbm_masses_host(self.h, self.stream())

    # -- adjoint (F64/F32 storage; periodic, walled or masked) ------------------
    def adjoint_workspace(self):
        """Device workspace of lbm_adjoint_step (allocated on first use)."""
        if getattr(self, "_adj_ws", None) is None:
            n = lbm_adjoint_workspace_bytes(self.params)
            if n == 0:
                raise LbmError(LBM_ENOTIMPL, "no adjoint for these parameters (needs F64/F32 storage)")
            self._adj_ws = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        return self._adj_ws

    def pops_like(self):
        """New [2, 9, ny, nx] tensor of the arithmetic type whose memory has the
        library's layout ([ny][colour][link][nx]): population states and
        adjoint buffers in this form pass to the library without a copy."""
        t = self.torch.empty((self.ny, 2, 9, self.nx), dtype=self.dtype, device=self.device)
        return t.permute(1, 2, 0, 3)

    def _is_lib_layout(self, t):
        n = self.nx
        return (tuple(t.shape) == (2, 9, self.ny, n) and t.dtype == self.dtype and t.device == self.device
                and tuple(t.stride()) == (9 * n, n, 18 * n, 1))

    def _in(self, t):
        """t ([2, 9, ny, nx]) in the library's memory layout (copied if needed)."""
        if self._is_lib_layout(t):
            return t
        out = self.pops_like()
        out.copy_(t)
        return out

    def _call_out(self, t, fn):
        """Run fn(pointer) that writes a [2, 9, ny, nx] buffer into t."""
        if self._is_lib_layout(t):
            fn(t.data_ptr())
        else:
            tmp = self.pops_like()
            fn(tmp.data_ptr())
            t.copy_(tmp)

    def adjoint_step(self, pops_t, adj_next, adj_out, dsigma=None, dforce=None):
        """adj_out = dL/dpops_t given adj_next = dL/dpops_{t+1}; adds dL/dsigma
        into dsigma (float64 device tensor of one element) and dL/dG_ext into
        dforce ([2, ny, nx]) when given.  States and adjoints are [2, 9, ny, nx]
        tensors (zero-copy when laid out as pops_like())."""
        ws = self.adjoint_workspace()
        S, L = self._in(pops_t), self._in(adj_next)
        self._call_out(adj_out, lambda ptr: lbm_adjoint_step(
            self.h, S.data_ptr(), L.data_ptr(), ptr, ws.data_ptr(), ws.numel(),
            None if dsigma is None else dsigma.data_ptr(), None if dforce is None else dforce.data_ptr(),
            self.stream()))

    def rhoN_adjoint(self, pops, dL_drhoN, adj_out):
        S, g = self._in(pops), dL_drhoN.contiguous()
        self._call_out(adj_out, lambda ptr: lbm_rhoN_adjoint(self.h, S.data_ptr(), g.data_ptr(), ptr,
                                                             self.stream()))

    def init_adjoint(self, adj0, dL_drhoN0):
        L = self._in(adj0)
        lbm_init_adjoint(self.h, self.rhoN0.data_ptr(), L.data_ptr(), dL_drhoN0.data_ptr(), self.stream())

    def set_pops(self, live, nxt):
        """Step from now on between the caller's buffers ``live`` (holding the
        current state) and ``nxt`` (receives the next step), both
        [2, 9, ny, nx] tensors laid out as pops_like() (F64/F32 storage)."""
        for t in (live, nxt):
            if not self._is_lib_layout(t):
                raise ValueError("set_pops needs [2, 9, ny, nx] buffers laid out as pops_like()")
        lbm_set_pops(self.h, live.data_ptr(), nxt.data_ptr())
        k = lbm_current_pops(self.h)
        # flat word views of the same memory, so live_pops() and friends follow
        self.pops[k] = live.permute(2, 0, 1, 3).reshape(-1)
        self.pops[1 - k] = nxt.permute(2, 0, 1, 3).reshape(-1)

    def live_words(self):
        """View [NW, ny, nx] of the live buffer (storage words, pull layout;
        the memory itself is [ny][NW][nx])."""
        return self.pops[lbm_current_pops(self.h)].view(self.ny, -1, self.nx).permute(1, 0, 2)

    def live_pops(self):
        """View [2, 9, ny, nx] of the live buffer (F64/F32 storage only)."""
        if self.storage not in ("f32", "f64"):
            raise ValueError("live_pops() needs F32/F64 storage; use live_words() for %s" % self.storage)
        return self.pops[lbm_current_pops(self.h)].view(self.ny, 2, 9, self.nx).permute(1, 2, 0, 3)

    @property
    def steps(self):
        return lbm_step_count(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batches of independent lattices
# ---------------------------------------------------------------------------

def lbm_batch_pops_bytes(plist):
    arr = (lbm_params * len(plist))(*plist)
    return load_library().lbm_batch_pops_bytes(arr, len(plist))


def lbm_batch_offsets(plist):
    lib = load_library()
    arr = (lbm_params * len(plist))(*plist)
    out = (ctypes.c_size_t * len(plist))()
    _check(lib, lib.lbm_batch_offsets(arr, len(plist), out))
    return list(out)


def lbm_batch_workspace_bytes(plist):
    arr = (lbm_params * len(plist))(*plist)
    return load_library().lbm_batch_workspace_bytes(arr, len(plist))


class Batch:
    """Independent lattices (all periodic or all walled) stepped together by one
    launch per step.

    lattices: list of (nx, ny, params, rhoN0); every lattice shares the
    storage format and the stencil radii.  ``state(k)`` is a view of lattice
    k's live population buffer ([2, 9, ny, nx], F32/F64 storage).
    """

    def __init__(self, lattices, storage="f32", device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the chromodynamic LBM step runs only on the HIP device")
        self.torch = torch
        self.device = torch.device(device)
        self.storage = storage
        self.dtype = torch.float64 if storage == "f64" else torch.float32
        self.shapes = [(nx, ny) for nx, ny, _, _ in lattices]
        self.plist = [make_params(nx, ny, storage, **dict(prm)) for nx, ny, prm, _ in lattices]
        lib = load_library()
        n = len(self.plist)
        arr = (lbm_params * n)(*self.plist)
        nbytes = lib.lbm_batch_pops_bytes(arr, n)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, lib.lbm_last_error().decode())
        self.offsets = lbm_batch_offsets(self.plist)
        self.pops = [torch.empty(nbytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        wsb = lib.lbm_batch_workspace_bytes(arr, n)
        self.ws = torch.zeros(wsb, dtype=torch.uint8, device=self.device)
        self.rhoN0 = [torch.as_tensor(np.asarray(r) if not torch.is_tensor(r) else r).to(
            device=self.device, dtype=self.dtype).contiguous() for _, _, _, r in lattices]
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.rhoN0])
        h = ctypes.c_void_p()
        _check(lib, lib.lbm_batch_init(arr, n, ptrs, self.pops[0].data_ptr(), self.pops[1].data_ptr(),
                                       self.ws.data_ptr(), wsb, self.stream(), ctypes.byref(h)))
        self.h = h
        self.lib = lib

    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def step(self, n=1):
        _check(self.lib, self.lib.lbm_batch_step(self.h, int(n), self.stream()))
        return self

    def autotune(self, steps_per_trial=5):
        scratch = self.torch.empty_like(self.pops[0])
        chosen = (ctypes.c_int32 * 2)()
        _check(self.lib, self.lib.lbm_batch_autotune(self.h, scratch.data_ptr(), scratch.numel(),
                                                     int(steps_per_trial), self.stream(), chosen))
        return chosen[0], chosen[1]

    def set_force(self, k, force):
        """Per-site force density of lattice k ([2, ny, nx], or None to remove it)."""
        t = None
        if force is not None:
            t = force if self.torch.is_tensor(force) else self.torch.as_tensor(np.asarray(force))
            t = t.to(device=self.device, dtype=self.dtype).contiguous()
            nx, ny = self.shapes[k]
            if tuple(t.shape) != (2, ny, nx):
                raise ValueError("force of lattice %d must have shape (2, %d, %d)" % (k, ny, nx))
        if not hasattr(self, "_forces"):
            self._forces = {}
        _check(self.lib, self.lib.lbm_batch_set_force(self.h, int(k), None if t is None else t.data_ptr(),
                                                      self.stream()))
        self._forces[k] = t          # kept alive while the batch uses it
        return self

    def set_solid(self, k, solid):
        """Mask of solid sites of lattice k ([ny, nx], nonzero = solid)."""
        t = self.torch
        nx, ny = self.shapes[k]
        m = solid if t.is_tensor(solid) else t.as_tensor(np.asarray(solid))
        m = (m != 0).to(device=self.device, dtype=t.uint8).contiguous()
        if tuple(m.shape) != (ny, nx):
            raise ValueError("mask of lattice %d must have shape (%d, %d)" % (k, ny, nx))
        n = self.lib.lbm_solid_workspace_bytes(ctypes.byref(self.plist[k]))
        ws = t.empty(max(n, 256), dtype=t.uint8, device=self.device)
        _check(self.lib, self.lib.lbm_batch_set_solid(self.h, int(k), m.data_ptr(), ws.data_ptr(), ws.numel(),
                                                      self.stream()))
        if not hasattr(self, "_solids"):
            self._solids = {}
        self._solids[k] = (m, ws)    # kept alive while the batch uses them
        return self

    def plan_info(self):
        info = (ctypes.c_int32 * 5)()
        _check(self.lib, self.lib.lbm_batch_plan_info(self.h, info))
        return dict(ntx=info[0], tycap=info[1], bins=info[2], items=info[3], max_cost=info[4])

    def state(self, k):
        nx, ny = self.shapes[k]
        live = self.lib.lbm_batch_current_pops(self.h)
        n = 18 * nx * ny * (8 if self.storage == "f64" else 4)
        return self.pops[live][self.offsets[k]:self.offsets[k] + n].view(self.dtype).view(ny, 2, 9, nx).permute(
            1, 2, 0, 3)

    def fields(self, k):
        t = self.torch
        nx, ny = self.shapes[k]
        out = {key: t.empty((ny, nx), dtype=self.dtype, device=self.device) for key in ("rho", "ux", "uy", "rhoN")}
        _check(self.lib, self.lib.lbm_batch_fields(self.h, int(k), out["rho"].data_ptr(), out["ux"].data_ptr(),
                                                   out["uy"].data_ptr(), out["rhoN"].data_ptr(), self.stream()))
        return out

    def masses(self, k):
        out = (ctypes.c_double * 2)()
        _check(self.lib, self.lib.lbm_batch_masses_host(self.h, int(k), out, self.stream()))
        return out[0], out[1]

    @property
    def steps(self):
        return self.lib.lbm_batch_step_count(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
