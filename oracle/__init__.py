"""FP64 CPU oracle of the chemical-potential multiphase LBM step -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle.so`` (built from ``lbm_oracle.c`` by
:func:`build`).  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product path never does.  It imports
nothing from the GPU package and the GPU package imports nothing from it.

Paper: Qin et al., "Spurious currents suppression by accurate difference schemes
in multiphase lattice Boltzmann method" (arXiv 2205.09186).  Citations name the
paper's sections, equations and tables.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

D2Q9, D3Q19 = 0, 1
CD2, CD4, CD6, E4, E8, OCFDS4, CFDS4, CFDS6, CFDS8, E6, E10 = range(11)
SCHEME_NAMES = {"CD2": CD2, "CD4": CD4, "CD6": CD6, "E4": E4, "E8": E8,
                "OCFDS4": OCFDS4, "CFDS4": CFDS4, "CFDS6": CFDS6, "CFDS8": CFDS8,
                "E6": E6, "E10": E10}

# Peng-Robinson constants used in the paper's simulations (Sec 2.2).
PR_A, PR_B, PR_R, PR_OMEGA = 2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over independent nodes)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("tau", C.c_double), ("Tr", C.c_double), ("k", C.c_double),
                ("kappa", C.c_double), ("scheme", C.c_int),
                ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
                ("omega", C.c_double), ("collision", C.c_int), ("s_e", C.c_double),
                ("s_eps", C.c_double), ("s_q", C.c_double), ("solid", C.c_void_p),
                ("mu_wall", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        P = C.POINTER(_Params)
        D = C.c_double
        L.orc_feq.argtypes = [C.c_int, D, D, D, D, dp]
        L.orc_lattice_info.argtypes = [C.c_int, ip, dp]
        L.orc_lattice_info.restype = C.c_int
        L.orc_collide_node.argtypes = [C.c_int, D, dp, D, D, D, dp]
        L.orc_collide_node_mrt.argtypes = [D, D, D, D, dp, D, D, D, dp]
        L.orc_mrt_matrix.argtypes = [dp, dp]
        L.orc_force.argtypes = [P, dp, dp, dp]
        L.orc_wall_density.argtypes = [P, dp, ip]
        L.orc_pr_alpha.argtypes = [D, D]; L.orc_pr_alpha.restype = D
        L.orc_pr_p0.argtypes = [D, D, D, D, D]; L.orc_pr_p0.restype = D
        L.orc_pr_mub.argtypes = [D, D, D, D, D]; L.orc_pr_mub.restype = D
        L.orc_pr_critical.argtypes = [D, D, D, C.POINTER(D), C.POINTER(D), C.POINTER(D)]
        L.orc_maxwell_mu.argtypes = [D, D, D, D, D, C.POINTER(D), C.POINTER(D)]
        L.orc_maxwell_area.argtypes = [D, D, D, D, D, C.POINTER(D), C.POINTER(D)]
        L.orc_compact_coeffs.argtypes = [C.c_int, dp]
        L.orc_cyclic_solve.argtypes = [C.c_int, D, dp, dp]
        L.orc_iso_stencil.argtypes = [C.c_int, C.c_int, ip, dp]
        L.orc_iso_stencil.restype = C.c_int
        L.orc_grad.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_lap.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_init.argtypes = [P, dp, dp]
        L.orc_step.argtypes = [P, dp, dp]
        L.orc_run.argtypes = [P, dp, dp, C.c_long]
        L.orc_macros.argtypes = [P, dp, dp, dp, dp, dp, C.c_void_p]
        L.orc_observables.argtypes = [P, dp, C.POINTER(D), C.POINTER(D)]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


# --------------------------------------------------------------------------- #
# Small helpers                                                                 #
# --------------------------------------------------------------------------- #

def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def lattice(lat: int):
    """(e[q,3] int, w[q]) of D2Q9 (Eq 2) or D3Q19."""
    e = np.zeros(19 * 3, np.int32)
    w = np.zeros(19, np.float64)
    q = lib().orc_lattice_info(lat, e, w)
    return e[: 3 * q].reshape(q, 3).copy(), w[:q].copy()


def feq(lat: int, rho: float, u) -> np.ndarray:
    """Equilibrium of Eq 6 at one node."""
    q = 9 if lat == D2Q9 else 19
    out = np.zeros(q)
    ux, uy, uz = (list(u) + [0.0, 0.0, 0.0])[:3]
    lib().orc_feq(lat, rho, ux, uy, uz, out)
    return out


def collide_node(lat: int, tau: float, f, F) -> np.ndarray:
    """SRT collision with EDM forcing at one node (Eq 1 with s_i = 1/tau, Eq 8)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    Fx, Fy, Fz = (list(F) + [0.0, 0.0, 0.0])[:3]
    lib().orc_collide_node(lat, tau, f, Fx, Fy, Fz, out)
    return out


def collide_node_mrt(tau: float, f, F, s_e: float = 0.0, s_eps: float = 0.0, s_q: float = 0.0) -> np.ndarray:
    """D2Q9 MRT collision with EDM forcing at one node (Eq 1, 3, 4, 5, 8);
    rates 0 select the values of Sec 2.1."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    Fx, Fy = (list(F) + [0.0, 0.0])[:2]
    lib().orc_collide_node_mrt(tau, s_e or 1.64, s_eps or 1.54, s_q or 1.7, f, Fx, Fy, 0.0, out)
    return out


def force(p: "Params", rho):
    """(F[dim, ...], mu_hat) of a density field (Eq 12, 15, 16) with p's scheme."""
    cp = p.c()
    r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    mu = np.zeros_like(r)
    F = np.zeros(3 * r.size)
    if lib().orc_force(C.byref(cp), r, mu, F):
        raise ValueError("invalid parameters")
    dim = 2 if p.lattice == D2Q9 else 3
    shape = np.shape(rho)
    return F[: dim * r.size].reshape((dim,) + shape), mu.reshape(shape)


def wall_density(p: "Params", rho):
    """(rho with the solid layers filled by Eq A.1, layer map) for p.solid:
    layer 0 fluid, 1..r the solid layers, -1 solid beyond them (Appendix)."""
    cp = p.c()
    r = np.array(rho, dtype=np.float64).reshape(-1)
    layer = np.zeros(r.size, np.int32)
    if lib().orc_wall_density(C.byref(cp), r, layer):
        raise ValueError("invalid parameters or no solid")
    return r.reshape(np.shape(rho)), layer.reshape(np.shape(rho))


def mrt_matrix():
    """(M of Eq 3, the oracle's numerical inverse of it)."""
    M = np.zeros(81)
    Mi = np.zeros(81)
    lib().orc_mrt_matrix(M, Mi)
    return M.reshape(9, 9), Mi.reshape(9, 9)


def pr_alpha(Tr: float, omega: float = PR_OMEGA) -> float:
    return lib().orc_pr_alpha(Tr, omega)


def pr_p0(rho: float, T: float, aa: float, b: float = PR_B, R: float = PR_R) -> float:
    """Pressure of Eq 14 with aa = a alpha(T)."""
    return lib().orc_pr_p0(rho, T, aa, b, R)


def pr_mub(rho: float, T: float, aa: float, b: float = PR_B, R: float = PR_R) -> float:
    """Bulk chemical potential psi'(rho) of Eq 15 (no gradient term)."""
    return lib().orc_pr_mub(rho, T, aa, b, R)


def pr_critical(a: float = PR_A, b: float = PR_B, R: float = PR_R):
    """(Tc, rho_c, p_c) of Eq 14 with alpha = 1."""
    Tc, rc, pc = C.c_double(), C.c_double(), C.c_double()
    rc_ = lib().orc_pr_critical(a, b, R, C.byref(Tc), C.byref(rc), C.byref(pc))
    if rc_:
        raise RuntimeError("critical point not found")
    return Tc.value, rc.value, pc.value


def maxwell(Tr: float, method: str = "mu", a: float = PR_A, b: float = PR_B,
            R: float = PR_R, omega: float = PR_OMEGA):
    """Coexistence densities (rho_g, rho_l) at T = Tr Tc by the Maxwell
    construction; method "mu" (equal mu and p) or "area" (equal areas in p-v)."""
    g, l = C.c_double(), C.c_double()
    fn = lib().orc_maxwell_mu if method == "mu" else lib().orc_maxwell_area
    if fn(Tr, a, b, R, omega, C.byref(g), C.byref(l)):
        raise ValueError(f"no coexistence at Tr={Tr}")
    return g.value, l.value


def compact_coeffs(scheme: int):
    """(alpha, a, b, c) of Eq 21 with beta = 0 for a compact scheme."""
    out = np.zeros(4)
    lib().orc_compact_coeffs(scheme, out)
    return tuple(out)


def cyclic_solve(alpha: float, d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float64)
    y = np.zeros_like(d)
    lib().orc_cyclic_solve(len(d), alpha, d, y)
    return y


def iso_stencil(dim: int, scheme: int):
    e = np.zeros(128 * 3, np.int32)
    w = np.zeros(128)
    n = lib().orc_iso_stencil(dim, scheme, e, w)
    if n < 0:
        raise ValueError(f"no isotropic stencil for scheme {scheme} in {dim}D")
    return e[: 3 * n].reshape(n, 3).copy(), w[:n].copy()


def _shape3(g):
    g = np.ascontiguousarray(g, dtype=np.float64)
    if g.ndim == 1:
        return g, 1, (1, 1, g.shape[0])
    if g.ndim == 2:
        return g, 2, (1,) + g.shape
    return g, 3, g.shape


def grad(g, scheme: int, dim: int | None = None) -> np.ndarray:
    """Discrete gradient of a periodic field (arrays indexed [z][y][x] or [y][x]).

    Returns an array of shape (dim,) + g.shape with components (x, y[, z])."""
    g, d0, (nz, ny, nx) = _shape3(g)
    dim = dim or max(d0, 2)
    out = np.zeros((3,) + g.shape)
    if lib().orc_grad(dim, nx, ny, nz, scheme, g.ravel(), out.reshape(-1)) != 0:
        raise ValueError(f"scheme {scheme} is not defined in {dim}D")
    return out[:dim]


def lap(g, scheme: int, dim: int | None = None) -> np.ndarray:
    g, d0, (nz, ny, nx) = _shape3(g)
    dim = dim or max(d0, 2)
    out = np.zeros(g.shape)
    if lib().orc_lap(dim, nx, ny, nz, scheme, g.ravel(), out.reshape(-1)) != 0:
        raise ValueError(f"scheme {scheme} is not defined in {dim}D")
    return out


# --------------------------------------------------------------------------- #
# Simulation                                                                    #
# --------------------------------------------------------------------------- #

@dataclass
class Params:
    lattice: int = D2Q9
    nx: int = 100
    ny: int = 100
    nz: int = 1
    tau: float = 1.0
    Tr: float = 0.8
    k: float = 0.25
    kappa: float = 0.01
    scheme: int = CD2
    a: float = PR_A
    b: float = PR_B
    R: float = PR_R
    omega: float = PR_OMEGA
    collision: int = 0          # 0 SRT, 1 MRT (D2Q9)
    s_e: float = 0.0
    s_eps: float = 0.0
    s_q: float = 0.0
    solid: np.ndarray | None = None   # uint8 per node (x fastest); nonzero = solid (Appendix)
    mu_wall: float = 0.0              # mu_hat on the solid layers

    @property
    def q(self) -> int:
        return 9 if self.lattice == D2Q9 else 19

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def c(self) -> _Params:
        sp = None
        if self.solid is not None:
            # keep a contiguous uint8 copy alive as long as this Params
            self._solid_buf = np.ascontiguousarray(self.solid, dtype=np.uint8).reshape(-1)
            assert self._solid_buf.size == self.n
            sp = self._solid_buf.ctypes.data
        return _Params(self.lattice, self.nx, self.ny, self.nz, self.tau, self.Tr, self.k,
                       self.kappa, self.scheme, self.a, self.b, self.R, self.omega, self.collision,
                       self.s_e, self.s_eps, self.s_q, sp, self.mu_wall)


class Sim:
    """Oracle simulation state: post-streaming populations f[q, N]."""

    def __init__(self, p: Params, rho0: np.ndarray):
        self.p = p
        self._cp = p.c()
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
        assert rho0.size == p.n
        self.f = np.zeros(p.q * p.n)
        self._w = np.zeros_like(self.f)
        if lib().orc_init(C.byref(self._cp), rho0, self.f):
            raise ValueError("invalid parameters or initial density")

    def step(self, n: int = 1) -> None:
        if lib().orc_run(C.byref(self._cp), self.f, self._w, int(n)):
            raise ValueError("oracle step failed")

    def macros(self, with_force: bool = False):
        p = self.p
        rho = np.zeros(p.n); vx = np.zeros(p.n); vy = np.zeros(p.n); vz = np.zeros(p.n)
        F = np.zeros(3 * p.n) if with_force else None
        fp = F.ctypes.data_as(C.c_void_p) if with_force else None
        if lib().orc_macros(C.byref(self._cp), self.f, rho, vx, vy, vz, fp):
            raise ValueError("oracle macros failed")
        shp = (p.nz, p.ny, p.nx) if p.lattice == D3Q19 else (p.ny, p.nx)
        out = [rho.reshape(shp), vx.reshape(shp), vy.reshape(shp), vz.reshape(shp)]
        if with_force:
            out.append(F.reshape((3,) + shp))
        return out

    def observables(self):
        u, m = C.c_double(), C.c_double()
        if lib().orc_observables(C.byref(self._cp), self.f, C.byref(u), C.byref(m)):
            raise ValueError("oracle observables failed")
        return u.value, m.value

    def populations(self) -> np.ndarray:
        return self.f.reshape(self.p.q, -1)
