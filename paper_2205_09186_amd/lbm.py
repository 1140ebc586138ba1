"""Python binding of the gfx950 library (``include/lbm.h``): argument marshalling only.

Every step of the method runs in the HIP kernels of ``liblbm.so``; PyTorch only
provides device memory (the workspace and device-side arrays) and the stream.
The binding refuses to run when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

D2Q9, D3Q19 = 0, 1
SRT, MRT = 0, 1
CD2, CD4, CD6, E4, E8, OCFDS4, CFDS4, CFDS6, CFDS8, E6, E10 = range(11)
SCHEMES = {"CD2": CD2, "CD4": CD4, "CD6": CD6, "E4": E4, "E8": E8, "OCFDS4": OCFDS4,
           "CFDS4": CFDS4, "CFDS6": CFDS6, "CFDS8": CFDS8, "E6": E6, "E10": E10}
LBM_OK, LBM_EINVAL, LBM_ENOSPC, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("tau", C.c_double), ("Tr", C.c_double), ("k", C.c_double), ("kappa", C.c_double),
                ("scheme", C.c_int), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
                ("omega", C.c_double), ("collision", C.c_int), ("s_e", C.c_double), ("s_eps", C.c_double),
                ("s_q", C.c_double), ("wall", C.c_int), ("mu_wall", C.c_double)]


_lib = None

# Every symbol the header declares, with (restype, argtypes).
_P = C.POINTER(lbm_params)
_D = C.POINTER(C.c_double)
SYMBOLS = {
    "lbm_workspace_bytes": (C.c_size_t, [_P]),
    "lbm_init": (C.c_int, [_P, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_init_wall": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_long]),
    "lbm_macros": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_spurious_max": (C.c_int, [C.c_void_p, _D, _D]),
    "lbm_populations": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_steps_done": (C.c_long, [C.c_void_p]),
    "lbm_state_bytes": (C.c_size_t, [C.c_void_p]),
    "lbm_save_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_load_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_step_timed": (C.c_int, [C.c_void_p, C.c_long, _D, C.c_int, C.POINTER(C.c_int)]),
    "lbm_phase_name": (C.c_char_p, [C.c_void_p, C.c_int]),
    "lbm_variant_name": (C.c_char_p, [C.c_void_p, C.c_int]),
    "lbm_num_variants": (C.c_int, [C.c_void_p]),
    "lbm_set_variant": (C.c_int, [C.c_void_p, C.c_int]),
    "lbm_free": (None, [C.c_void_p]),
    "lbm_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_critical": (C.c_int, [_P, _D, _D, _D]),
    "lbm_batch_workspace_bytes": (C.c_size_t, [_P, C.c_int]),
    "lbm_batch_init": (C.c_int, [_P, C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    "lbm_batch_set_grid": (C.c_int, [C.c_void_p, C.c_int]),
    "lbm_batch_max_grid": (C.c_int, [C.c_void_p]),
    "lbm_batch_set_block": (C.c_int, [C.c_void_p, C.c_int]),
    "lbm_batch_block": (C.c_int, [C.c_void_p]),
    "lbm_batch_set_form": (C.c_int, [C.c_void_p, C.c_int]),
    "lbm_batch_form": (C.c_int, [C.c_void_p]),
    "lbm_batch_launch_mode": (C.c_char_p, [C.c_void_p]),
    "lbm_batch_run": (C.c_int, [C.c_void_p, C.c_long, C.c_long, C.c_double, C.c_long, C.POINTER(C.c_int),
                                C.POINTER(C.c_long), _D]),
    "lbm_batch_instance": (C.c_void_p, [C.c_void_p, C.c_int]),
    "lbm_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_batch_free": (None, [C.c_void_p]),
    "mlp_param_count": (C.c_int, []),
    "mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mlp_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.c_float,
                           C.c_float, C.c_float, C.c_void_p]),
    "mlp_field": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), _P, C.c_double, C.c_double, C.c_double, C.c_double,
                            C.POINTER(C.c_float), C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "lbm_sum_scratch_bytes": (C.c_size_t, [C.c_long]),
    "lbm_sum": (C.c_int, [C.c_void_p, C.c_long, C.c_void_p, _D, C.c_void_p]),
    "lbm_interface_mass": (C.c_int, [C.c_void_p, C.c_long, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                     C.c_void_p]),
    "lbm_sum_static_max": (C.c_size_t, []),
    "lbm_sum_static": (C.c_int, [C.c_void_p, C.c_long, _D, C.c_void_p]),
    "lbm_probe_copy": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "lbm_coexistence": (C.c_int, [_P, _D, _D]),
    "lbm_eos": (C.c_int, [_P, C.c_void_p, C.c_long, C.c_void_p, C.c_void_p]),
    "lbm_force": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}


def lib():
    """Load liblbm.so (fails loudly if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # load PyTorch's HIP runtime first so the library binds to the same
        # runtime instance that owns the workspace memory and the streams
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _err(ctx=None) -> str:
    m = lib().lbm_last_error(ctx)
    return m.decode() if m else ""


def _check(code: int, ctx=None):
    if code != LBM_OK:
        raise LbmError(code, _err(ctx))


@dataclass
class Params:
    lattice: int = D2Q9
    nx: int = 100
    ny: int = 100
    nz: int = 1
    tau: float = 1.0
    Tr: float = 0.8
    k: float = 0.16
    kappa: float = 0.004
    scheme: int = CD4
    a: float = 0.0
    b: float = 0.0
    R: float = 0.0
    omega: float = 0.0
    collision: int = SRT       # SRT or MRT (D2Q9, Eq 1, 3, 5)
    s_e: float = 0.0           # MRT rates; 0 selects the values of Sec 2.1
    s_eps: float = 0.0
    s_q: float = 0.0
    wall: int = 0              # 1: solid nodes passed to Simulation(..., solid=) (Appendix)
    mu_wall: float = 0.0       # mu_hat of the solid layers

    def c(self) -> lbm_params:
        return lbm_params(self.lattice, self.nx, self.ny, self.nz, self.tau, self.Tr, self.k, self.kappa,
                          self.scheme, self.a, self.b, self.R, self.omega, self.collision, self.s_e, self.s_eps,
                          self.s_q, self.wall, self.mu_wall)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def q(self) -> int:
        return 9 if self.lattice == D2Q9 else 19

    @property
    def shape(self):
        return (self.ny, self.nx) if self.lattice == D2Q9 else (self.nz, self.ny, self.nx)


def workspace_bytes(p: Params) -> int:
    cp = p.c()
    return int(lib().lbm_workspace_bytes(C.byref(cp)))


def critical(p: Params | None = None):
    cp = (p or Params()).c()
    Tc, rc, pc = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_critical(C.byref(cp), C.byref(Tc), C.byref(rc), C.byref(pc)))
    return Tc.value, rc.value, pc.value


def eos(rho, Tr: float, p: Params | None = None):
    """(p0, psi') of the Peng-Robinson EOS (Eq 14, 15; not scaled by k) at
    host densities rho, T = Tr Tc."""
    q = Params(**{**(p or Params()).__dict__, "Tr": Tr})
    cp = q.c()
    r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    p0, mu = np.empty_like(r), np.empty_like(r)
    _check(lib().lbm_eos(C.byref(cp), r.ctypes.data, r.size, p0.ctypes.data, mu.ctypes.data))
    return p0.reshape(np.shape(rho)), mu.reshape(np.shape(rho))


def coexistence(Tr: float, p: Params | None = None):
    """Maxwell-construction (rho_g, rho_l) at reduced temperature Tr."""
    q = Params(**{**(p or Params()).__dict__, "Tr": Tr})
    cp = q.c()
    g, l = C.c_double(), C.c_double()
    _check(lib().lbm_coexistence(C.byref(cp), C.byref(g), C.byref(l)))
    return g.value, l.value


class _View:
    """Observables of a context owned elsewhere (an instance of a batch)."""

    def __init__(self, ctx, p: Params, device, owner):
        import torch
        self.ctx, self.p, self.device, self.torch, self._owner = ctx, p, device, torch, owner


class Simulation:
    """One lattice on one GPU: a caller-owned torch workspace, a torch stream."""

    def __init__(self, p: Params, rho0, device: str = "cuda:0", stream=None, solid=None):
        """solid: optional uint8 mask shaped like the grid (nonzero = solid
        node) for the wetting boundary; needs p.wall = 1."""
        import torch
        self.p = p
        self.torch = torch
        self.device = torch.device(device)
        self._cp = p.c()
        nbytes = workspace_bytes(p)
        if nbytes == 0:
            _check(LBM_EINVAL)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        if isinstance(rho0, torch.Tensor) and rho0.is_cuda:
            r = rho0.to(torch.float64).contiguous()
            self._rho0_keep = r
            ptr, on_dev = C.c_void_p(r.data_ptr()), 1
        else:
            r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
            if r.size != p.n:
                raise ValueError("rho0 has the wrong size")
            self._rho0_keep = r
            ptr, on_dev = r.ctypes.data_as(C.c_void_p), 0
        if solid is None:
            code = lib().lbm_init(C.byref(self._cp), ptr, on_dev, C.c_void_p(self.ws.data_ptr()), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        else:
            if on_dev:
                m = torch.as_tensor(solid, device=self.device).to(torch.uint8).contiguous().reshape(-1)
                sptr = C.c_void_p(m.data_ptr())
            else:
                m = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
                sptr = m.ctypes.data_as(C.c_void_p)
            if (m.numel() if on_dev else m.size) != p.n:
                raise ValueError("solid has the wrong size")
            self._solid_keep = m
            code = lib().lbm_init_wall(C.byref(self._cp), ptr, sptr, on_dev, C.c_void_p(self.ws.data_ptr()),
                                       nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        _check(code)
        self.ctx = ctx

    def step(self, n: int = 1) -> None:
        _check(lib().lbm_step(self.ctx, int(n)), self.ctx)

    def step_timed(self, n: int):
        """Run n steps timing each phase with HIP events: [(name, mean ms per step)]."""
        ms = (C.c_double * 16)()
        npk = C.c_int()
        _check(lib().lbm_step_timed(self.ctx, int(n), ms, 16, C.byref(npk)), self.ctx)
        return [(lib().lbm_phase_name(self.ctx, k).decode(), ms[k]) for k in range(npk.value)]

    @property
    def num_variants(self) -> int:
        return int(lib().lbm_num_variants(self.ctx))

    def set_variant(self, v: int) -> None:
        _check(lib().lbm_set_variant(self.ctx, int(v)), self.ctx)

    def variant_name(self, v: int) -> str:
        """What launch variant v is, e.g. 'tile 64x16 z64 mf'."""
        return lib().lbm_variant_name(self.ctx, int(v)).decode()

    def tune(self, steps: int = 5, rounds: int = 1, restore: bool = False):
        """Time every launch variant of the step kernel on this grid and keep
        the fastest.  Each round takes every variant in turn for one untimed
        and `steps` timed steps; a variant's time is its best round, so drift
        over the rounds does not favour the variants timed last.  The state
        advances by (steps + 1) * variants * rounds steps, or with
        restore=True returns to where it was (a device state image, which
        also restores the step count).  Returns {variant: ms per step}."""
        img = self.save_state(device=True) if restore else None
        res = {}
        for r in range(rounds):
            for v in range(self.num_variants):
                self.set_variant(v)
                self.step_timed(1)
                t = sum(t for _, t in self.step_timed(steps))
                res[v] = t if r == 0 else min(res[v], t)
        best = min(res, key=res.get)
        self.set_variant(best)
        if img is not None:
            self.load_state(img)
        return res

    @property
    def steps_done(self) -> int:
        return int(lib().lbm_steps_done(self.ctx))

    def save_state(self, device: bool = False):
        """State image (lbm_save_state): a host numpy uint8 array, or with
        device=True a torch uint8 tensor on the context's device."""
        nbytes = int(lib().lbm_state_bytes(self.ctx))
        if device:
            img = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
            _check(lib().lbm_save_state(self.ctx, C.c_void_p(img.data_ptr()), 1), self.ctx)
        else:
            img = np.empty(nbytes, np.uint8)
            _check(lib().lbm_save_state(self.ctx, img.ctypes.data_as(C.c_void_p), 0), self.ctx)
        return img

    def load_state(self, img) -> None:
        """Restore an image from save_state (host array or device tensor)."""
        if hasattr(img, "data_ptr") and img.is_cuda:
            _check(lib().lbm_load_state(self.ctx, C.c_void_p(img.data_ptr()), 1), self.ctx)
        else:
            a = np.ascontiguousarray(img, dtype=np.uint8)
            _check(lib().lbm_load_state(self.ctx, a.ctypes.data_as(C.c_void_p), 0), self.ctx)

    def macros(self):
        """(rho, vx, vy, vz) host arrays shaped like the grid (vz None in 2D)."""
        return _macros(self)

    def macros_device(self):
        """(rho, vx, vy[, vz]) as torch float64 tensors on the device."""
        t = self.torch
        k = 4 if self.p.lattice == D3Q19 else 3
        out = [t.empty(self.p.n, dtype=t.float64, device=self.device) for _ in range(k)]
        ptrs = [C.c_void_p(a.data_ptr()) for a in out] + ([None] if k == 3 else [])
        _check(lib().lbm_macros(self.ctx, *ptrs, 1), self.ctx)
        return [a.view(self.p.shape) for a in out]

    def spurious_max(self, raise_on_nonfinite: bool = False):
        """(U = max |v|, total mass, status code)."""
        return _spurious(self, raise_on_nonfinite)

    def force(self):
        """(F[dim, *shape], mu_hat[*shape]) of the current state as host arrays
        (Eq 12, 16, with the context's scheme)."""
        dim = 3 if self.p.lattice == D3Q19 else 2
        F = np.empty(dim * self.p.n)
        mu = np.empty(self.p.n)
        _check(lib().lbm_force(self.ctx, F.ctypes.data, mu.ctypes.data, 0), self.ctx)
        return F.reshape((dim,) + self.p.shape), mu.reshape(self.p.shape)

    def gradient(self, field):
        """(grad[dim, *shape], lap[*shape]) of a field with the context's scheme,
        as device tensors (the field is copied to the device if needed)."""
        t = self.torch
        f = t.as_tensor(np.ascontiguousarray(field, dtype=np.float64).reshape(-1) if not t.is_tensor(field)
                        else field.reshape(-1)).to(self.device, t.float64).contiguous()
        dim = 3 if self.p.lattice == D3Q19 else 2
        g = t.empty(dim * self.p.n, dtype=t.float64, device=self.device)
        lap = t.empty(self.p.n, dtype=t.float64, device=self.device)
        _check(lib().lbm_gradient(self.ctx, C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr()),
                                  C.c_void_p(lap.data_ptr())), self.ctx)
        t.cuda.current_stream().synchronize()
        return g.view((dim,) + self.p.shape), lap.view(self.p.shape)

    def populations(self) -> np.ndarray:
        return _populations(self)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            lib().lbm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _macros(obj):
    p = obj.p
    out = [np.empty(p.n) for _ in range(4 if p.lattice == D3Q19 else 3)]
    ptrs = [a.ctypes.data_as(C.c_void_p) for a in out] + ([None] if p.lattice == D2Q9 else [])
    _check(lib().lbm_macros(obj.ctx, *ptrs, 0), obj.ctx)
    res = [a.reshape(p.shape) for a in out]
    return tuple(res) if p.lattice == D3Q19 else (res[0], res[1], res[2], None)


def _spurious(obj, raise_on_nonfinite=False):
    u, m = C.c_double(), C.c_double()
    code = lib().lbm_spurious_max(obj.ctx, C.byref(u), C.byref(m))
    if code not in (LBM_OK, LBM_ENONFINITE) or (raise_on_nonfinite and code != LBM_OK):
        _check(code, obj.ctx)
    return u.value, m.value, code


def _populations(obj):
    f = np.empty(obj.p.q * obj.p.n)
    _check(lib().lbm_populations(obj.ctx, f.ctypes.data_as(C.c_void_p), 0), obj.ctx)
    return f.reshape(obj.p.q, -1)


_View.macros = _macros
_View.spurious_max = _spurious
_View.populations = _populations
_View.steps_done = property(lambda self: int(lib().lbm_steps_done(self.ctx)))
_View.save_state = Simulation.save_state
_View.load_state = Simulation.load_state

RUNNING, CONVERGED, DIVERGED = 0, 1, 2


BATCH_PERSISTENT, BATCH_PHASES = 0, 1


class Batch:
    """Uneven D2Q9 instances stepped together, by the cooperative persistent
    kernel (form BATCH_PERSISTENT) or by one launch per phase (BATCH_PHASES)."""

    def __init__(self, params, rho0s, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = list(params)
        n = len(self.params)
        self._cps = (lbm_params * n)(*[p.c() for p in self.params])
        nbytes = int(lib().lbm_batch_workspace_bytes(self._cps, n))
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, _err(None))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._rho = [np.ascontiguousarray(r, dtype=np.float64).reshape(-1) for r in rho0s]
        ptrs = (C.c_void_p * n)(*[r.ctypes.data for r in self._rho])
        h = C.c_void_p()
        code = lib().lbm_batch_init(self._cps, ptrs, n, C.c_void_p(self.ws.data_ptr()), nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if code != LBM_OK:
            raise LbmError(code, _err(None))
        self.h = h
        self.n = n

    @property
    def max_grid(self) -> int:
        return int(lib().lbm_batch_max_grid(self.h))

    def set_grid(self, wg: int) -> None:
        code = lib().lbm_batch_set_grid(self.h, int(wg))
        if code != LBM_OK:
            raise LbmError(code, lib().lbm_batch_last_error(self.h).decode())

    @property
    def block(self) -> int:
        return int(lib().lbm_batch_block(self.h))

    def set_block(self, nodes: int) -> None:
        """Node-block size (256, 512, 1024); resets the workgroup count."""
        code = lib().lbm_batch_set_block(self.h, int(nodes))
        if code != LBM_OK:
            raise LbmError(code, lib().lbm_batch_last_error(self.h).decode())

    @property
    def form(self) -> int:
        return int(lib().lbm_batch_form(self.h))

    def set_form(self, form: int) -> None:
        """BATCH_PERSISTENT or BATCH_PHASES (bitwise the same states)."""
        code = lib().lbm_batch_set_form(self.h, int(form))
        if code != LBM_OK:
            raise LbmError(code, lib().lbm_batch_last_error(self.h).decode())

    @property
    def launch_mode(self) -> str:
        return lib().lbm_batch_launch_mode(self.h).decode()

    def run(self, nsteps: int, check_every: int = 100, tol: float = 1e-10, chunk: int = 1000, progress=None):
        """Advance; returns (status[n], steps[n], U[n]) numpy arrays.  With a
        progress callback the run is issued chunk by chunk and the callback
        receives (steps issued, status array) after each."""
        st = (C.c_int * self.n)()
        sp = (C.c_long * self.n)()
        um = (C.c_double * self.n)()
        done = 0
        while True:
            todo = nsteps - done if progress is None else min(chunk, nsteps - done)
            code = lib().lbm_batch_run(self.h, int(todo), int(check_every), float(tol), int(chunk), st, sp, um)
            if code != LBM_OK:
                raise LbmError(code, lib().lbm_batch_last_error(self.h).decode())
            done += todo
            status = np.array(st[:])
            if progress is not None:
                progress(done, status)
            if done >= nsteps or not (status == RUNNING).any():
                break
        return status, np.array(sp[:]), np.array(um[:])

    def instance(self, i: int):
        ctx = lib().lbm_batch_instance(self.h, int(i))
        return _View(C.c_void_p(ctx), self.params[i], self.device, self)

    def tune(self, steps: int = 50, blocks=(256, 512, 1024), forms=(BATCH_PERSISTENT, BATCH_PHASES)):
        """Time the launch for every node-block size and, for each, the
        persistent form with the most resident workgroups and a half and a
        quarter of them, and the phase form (the state advances); keep the
        fastest.  Each combination runs once untimed (its launch graph is
        captured then) and once timed.
        Returns {"block/workgroups": ms per step}, workgroups "phases" for the
        phase form."""
        import time
        res = {}
        for bn in blocks:
            self.set_block(bn)
            mg = self.max_grid
            cands = []
            if BATCH_PERSISTENT in forms:
                cands += [(BATCH_PERSISTENT, wg) for wg in sorted({mg, max(1, mg // 2), max(1, mg // 4)})]
            if BATCH_PHASES in forms:
                cands.append((BATCH_PHASES, mg))
            for form, wg in cands:
                self.set_form(form)
                self.set_grid(wg)
                self.run(steps, check_every=10 ** 9, tol=0.0, chunk=steps)
                if self.form != form:   # the runtime refused the persistent form
                    continue
                self.torch.cuda.synchronize()
                t0 = time.perf_counter()
                self.run(steps, check_every=10 ** 9, tol=0.0, chunk=steps)
                res[f"{bn}/{'phases' if form == BATCH_PHASES else wg}"] = (time.perf_counter() - t0) * 1e3 / steps
        best = min(res, key=res.get)
        bs, ws = best.split("/")
        self.set_block(int(bs))
        if ws == "phases":
            self.set_form(BATCH_PHASES)
        else:
            self.set_form(BATCH_PERSISTENT)
            self.set_grid(int(ws))
        return res

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
