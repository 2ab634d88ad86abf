"""CPU FP64 oracle for the hybrid multi-time-step FEM/LBM coupling.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package; the product path
(the HIP library and its Python binding) never does.

The per-node / per-element arithmetic lives in plain C (``lbm_oracle.c``,
``fem_oracle.c``, built with ``gcc -O2 -ffp-contract=off``); the control flow
of the coupling algorithm (Algorithm 1) is written out in ``hybrid.py``.
Everything is FP64.  It shares no code, header or table with the HIP path;
the only common module is the seeded input generator
``paper_1601_02708_amd.inputs`` (which holds no part of the method).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

c_int = ctypes.c_int
c_double = ctypes.c_double
c_long = ctypes.c_long
c_void_p = ctypes.c_void_p


class OrcLattice(ctypes.Structure):
    _fields_ = [("N", c_int), ("periodic_x", c_int), ("periodic_y", c_int),
                ("tau", c_double), ("solid", c_void_p), ("vx", c_void_p), ("vy", c_void_p),
                ("k", c_void_p), ("kval", c_double), ("bc_kind", c_void_p), ("clamp", c_int),
                ("kappa_s", c_double), ("c_sat", c_double), ("work_f", c_void_p), ("work_unknown", c_void_p),
                ("wall_nx", c_void_p), ("wall_ny", c_void_p)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        srcs = [os.path.join(_HERE, s) for s in _build.SOURCES]
        if (not os.path.exists(path)) or any(os.path.getmtime(s) > os.path.getmtime(path) for s in srcs):
            _build.build()
        L = ctypes.CDLL(path)
        P = c_void_p
        sig = {
            "orc_d2q9": (None, [P, P, P, P]),
            "orc_set_threads": (None, [c_int]),
            "orc_get_threads": (c_int, []),
            "orc_feq": (None, [c_double, c_double, c_double, P]),
            "orc_perimeter_slot": (c_int, [c_int, c_int, c_int]),
            "orc_perimeter_node": (None, [c_int, c_int, P, P]),
            "orc_lbm_init": (None, [P, P, P]),
            "orc_stream": (None, [P, P, P, P]),
            "orc_maxent_dirichlet": (c_int, [P, ctypes.c_uint, c_double, c_int]),
            "orc_maxent_neumann": (c_int, [P, ctypes.c_uint, c_int, c_int, c_double, P]),
            "orc_maxent_neumann_normal": (c_int, [P, ctypes.c_uint, c_double, c_double, c_double, P]),
            "orc_apply_wall_closure": (c_long, [P, P, P]),
            "orc_apply_bc": (c_long, [P, P, P, P, P]),
            "orc_collide": (None, [P, P, P]),
            "orc_lbm_substep": (c_long, [P, P, P, P]),
            "orc_lbm_adjoint_substep": (c_int, [P, P, P, P, P, P, P]),
            "orc_concentration": (None, [P, P, P]),
            "orc_h_function": (c_double, [P, P]),
            "orc_supg_chi": (c_double, [c_double]),
            "orc_fem_element": (None, [c_double, c_double, c_double, c_int, P, P, P, P, P]),
            "orc_fem_assemble": (None, [c_int, c_double, c_double, c_double, c_double, c_int, P, P, P]),
            "orc_band_dirichlet_rows": (None, [c_int, P, P, c_int]),
            "orc_band_matvec": (None, [c_int, P, P, P]),
            "orc_band_to_dense": (None, [c_int, P, P]),
            "orc_band_lu": (c_int, [c_int, P, P]),
            "orc_band_solve": (None, [c_int, P, P, P]),
            "orc_fem_interpolate": (c_double, [c_int, c_double, P, c_double, c_double]),
            "orc_fine_to_coarse": (c_double, [c_int, P, P, c_double, c_double]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# lattice constants and single-node pieces
# ----------------------------------------------------------------------------

def d2q9():
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9)
    opp = np.zeros(9, np.int32)
    lib().orc_d2q9(_p(ex), _p(ey), _p(w), _p(opp))
    return ex, ey, w, opp


def set_threads(n):
    """Threads of the oracle's row-parallel lattice loops (n >= 1; the
    default is OpenMP's, OMP_NUM_THREADS when set).  Results do not depend
    on it."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def sound_speed_sq():
    """c_s^2 of the D2Q9 lattice as its second velocity moment,
    sum_i w_i e_ix^2 (Sec. 4.1: c_s = dx / (sqrt(3) dt), so 1/3 in lattice
    units)."""
    ex, _, w, _ = d2q9()
    return float(np.sum(w * ex.astype(np.float64) ** 2))


def relaxation_time(D, tau=None):
    """BGK relaxation time of the lattice-unit problem (fine step 1,
    spacing 1): tau = 1/2 + D / c_s^2 (Sec. 4.1, the relation between the
    diffusion coefficient and the relaxation time), unless an explicit
    ``tau`` overrides it."""
    if tau is not None:
        return float(tau)
    return 0.5 + float(D) / sound_speed_sq()


def feq(u, vx, vy):
    out = np.zeros(9)
    lib().orc_feq(float(u), float(vx), float(vy), _p(out))
    return out


def maxent_dirichlet(f, unknown: int, up: float, clamp: bool = False):
    f = _f64(f).copy()
    inf = lib().orc_maxent_dirichlet(_p(f), int(unknown), float(up), int(clamp))
    return f, int(inf)


def maxent_neumann(f, unknown: int, sx: int, sy: int, qp: float, fstar_self):
    f = _f64(f).copy()
    fs = _f64(fstar_self)
    inf = lib().orc_maxent_neumann(_p(f), int(unknown), int(sx), int(sy), float(qp), _p(fs))
    return f, int(inf)


def maxent_neumann_normal(f, unknown: int, nx: float, ny: float, qp: float, fstar_self):
    """eq. (LBM_Neu) for a real unit outward normal (nx, ny)."""
    f = _f64(f).copy()
    fs = _f64(fstar_self)
    inf = lib().orc_maxent_neumann_normal(_p(f), int(unknown), float(nx), float(ny), float(qp), _p(fs))
    return f, int(inf)


def perimeter_slot(N, i, j):
    return lib().orc_perimeter_slot(N, i, j)


def perimeter_nodes(N):
    """(i, j) integer arrays of the 4(N-1) perimeter slots in slot order."""
    P = 4 * (N - 1)
    ii = np.zeros(P, np.int64)
    jj = np.zeros(P, np.int64)
    a = ctypes.c_int()
    b = ctypes.c_int()
    for p in range(P):
        lib().orc_perimeter_node(N, p, ctypes.addressof(a), ctypes.addressof(b))
        ii[p], jj[p] = a.value, b.value
    return ii, jj


# ----------------------------------------------------------------------------
# lattice sweeps
# ----------------------------------------------------------------------------

class Lattice:
    """An N x N D2Q9 lattice with its fields (all FP64 on the host)."""

    def __init__(self, N, tau, vx, vy, solid=None, k=0.0, bc_kind=None,
                 periodic_x=False, periodic_y=False, clamp=False, kappa_s=0.0, c_sat=0.0, wall_normals=None):
        self.N = int(N)
        self.tau = float(tau)
        self.vx = _f64(vx).reshape(N, N)
        self.vy = _f64(vy).reshape(N, N)
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(N, N)
        if np.isscalar(k):
            self.kfield, self.kval = None, float(k)
        else:
            self.kfield, self.kval = _f64(k).reshape(N, N), 0.0
        self.bc_kind = None if bc_kind is None else np.ascontiguousarray(bc_kind, dtype=np.int8)
        # wall_normals: [2, N, N] unit outward normals of the fluid domain
        # at solid walls (the maximum-entropy zero-flux closure replaces
        # bounce-back there), or None
        if wall_normals is None:
            self.wall_nx = self.wall_ny = None
        else:
            wn = _f64(wall_normals).reshape(2, N, N)
            self.wall_nx, self.wall_ny = np.ascontiguousarray(wn[0]), np.ascontiguousarray(wn[1])
        # scratch of one step, allocated once per lattice (no values carry
        # over between steps)
        self._work_f = np.empty((9, self.N, self.N))
        self._work_unknown = np.empty((self.N, self.N), np.uint16)
        self.s = OrcLattice(self.N, int(periodic_x), int(periodic_y), self.tau, _p(self.solid),
                            _p(self.vx), _p(self.vy), _p(self.kfield), self.kval, _p(self.bc_kind),
                            int(clamp), float(kappa_s), float(c_sat), _p(self._work_f), _p(self._work_unknown),
                            _p(self.wall_nx), _p(self.wall_ny))
        self.kappa_s, self.c_sat = float(kappa_s), float(c_sat)

    @property
    def ptr(self):
        return ctypes.addressof(self.s)

    def init(self, u0):
        u0 = _f64(u0).reshape(self.N, self.N)
        out = np.zeros((9, self.N, self.N))
        lib().orc_lbm_init(self.ptr, _p(u0), _p(out))
        return out

    def substep(self, fsrc, bc_value=None, out=None):
        """One fine step from fsrc into a new array, or into ``out`` (a
        C-contiguous FP64 array of fsrc's shape that is not fsrc)."""
        fsrc = _f64(fsrc)
        if bc_value is None:
            bc_value = np.zeros(4 * (self.N - 1))
        bc_value = _f64(bc_value)
        if out is None:
            out = np.empty_like(fsrc)
        elif out is fsrc or out.shape != fsrc.shape or out.dtype != np.float64 or not out.flags.c_contiguous:
            raise ValueError("out must be a separate C-contiguous FP64 array of the state's shape")
        inf = lib().orc_lbm_substep(self.ptr, _p(fsrc), _p(out), _p(bc_value))
        return out, int(inf)

    def adjoint_substep(self, fsrc, bc_value, lam_in):
        """Reverse mode of substep(fsrc, bc_value): returns (dJ/df*(t),
        dJ/du^p per perimeter slot, dJ/dk per node) for lam_in = dJ/df*(t+1).
        All perimeter slots must be Dirichlet."""
        fsrc = _f64(fsrc)
        bc_value = _f64(np.zeros(4 * (self.N - 1)) if bc_value is None else bc_value)
        lam_in = _f64(lam_in)
        lam_out = np.empty_like(lam_in)
        gbc = np.zeros(4 * (self.N - 1))
        gk = np.zeros((self.N, self.N))
        rc = lib().orc_lbm_adjoint_substep(self.ptr, _p(fsrc), _p(bc_value), _p(lam_in), _p(lam_out), _p(gbc),
                                           _p(gk))
        if rc != 0:
            raise ValueError("adjoint supports Dirichlet perimeter slots only")
        return lam_out, gbc, gk

    def stream(self, fsrc):
        fsrc = _f64(fsrc)
        f = np.empty_like(fsrc)
        unk = np.zeros((self.N, self.N), np.uint16)
        lib().orc_stream(self.ptr, _p(fsrc), _p(f), _p(unk))
        return f, unk

    def collide(self, f):
        f = _f64(f)
        out = np.empty_like(f)
        lib().orc_collide(self.ptr, _p(f), _p(out))
        return out

    def concentration(self, fstar):
        fstar = _f64(fstar)
        u = np.empty((self.N, self.N))
        lib().orc_concentration(self.ptr, _p(fstar), _p(u))
        return u

    def h_function(self, f):
        return lib().orc_h_function(self.ptr, _p(_f64(f)))


# ----------------------------------------------------------------------------
# coarse FEM
# ----------------------------------------------------------------------------

def supg_chi(a):
    return lib().orc_supg_chi(float(a))


def fem_element(h, D, k, supg, vn):
    vn = _f64(vn).reshape(4, 2)
    mats = [np.zeros((4, 4)) for _ in range(4)]
    lib().orc_fem_element(float(h), float(D), float(k), int(supg), _p(vn), *[_p(m) for m in mats])
    return tuple(mats)


def _ldab(M):
    return 2 * (M + 2) + (M + 2) + 1


def fem_matrices(M, L, D, k, dt, supg, vnodes):
    """Band arrays of A = (M+Ms) + dt/2 (K+Ks) and B = (M+Ms) - dt/2 (K+Ks)."""
    n = (M + 1) ** 2
    vnodes = _f64(vnodes).reshape(n, 2)
    a = np.zeros(n * _ldab(M))
    b = np.zeros(n * _ldab(M))
    lib().orc_fem_assemble(M, float(L), float(D), float(k), float(dt), int(supg), _p(vnodes), _p(a), _p(b))
    return a, b


def band_to_dense(M, band):
    n = (M + 1) ** 2
    out = np.zeros((n, n))
    lib().orc_band_to_dense(M, _p(_f64(band)), _p(out))
    return out


def band_solve(M, A, b):
    """Solve a dense matrix whose nonzeros lie within M + 2 diagonals of the
    main one through the oracle's band LU (test helper)."""
    n = (M + 1) ** 2
    kl = ku = M + 2
    ldab = _ldab(M)
    ab = np.zeros(n * ldab)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[j * ldab + kl + ku + i - j] = A[i, j]
    ipiv = np.zeros(n, np.int32)
    rc = lib().orc_band_lu(M, _p(ab), _p(ipiv))
    if rc != 0:
        raise RuntimeError("singular")
    x = _f64(b).copy()
    lib().orc_band_solve(M, _p(ab), _p(ipiv), _p(x))
    return x


class FemStepper:
    """One trapezoidal step of the Q1 system with fixed strong-Dirichlet rows:
    A d1 = B d0 on free rows, d1 = prescribed value on Dirichlet rows."""

    def __init__(self, M, L, D, k, dt, supg, vnodes, dirichlet_rows):
        self.M = M
        self.n = (M + 1) ** 2
        self.rows = np.ascontiguousarray(np.sort(np.asarray(dirichlet_rows)), dtype=np.int32)
        self.a, self.b = fem_matrices(M, L, D, k, dt, supg, vnodes)
        lib().orc_band_dirichlet_rows(M, _p(self.a), _p(self.rows), len(self.rows))
        self.ipiv = np.zeros(self.n, np.int32)
        rc = lib().orc_band_lu(M, _p(self.a), _p(self.ipiv))
        if rc != 0:
            raise RuntimeError(f"singular coarse matrix (column {rc - 1})")

    def rhs(self, d0):
        y = np.zeros(self.n)
        lib().orc_band_matvec(self.M, _p(self.b), _p(_f64(d0)), _p(y))
        return y

    def step(self, d0, dirichlet_values):
        """dirichlet_values: array aligned with the sorted Dirichlet rows."""
        y = self.rhs(d0)
        y[self.rows] = dirichlet_values
        lib().orc_band_solve(self.M, _p(self.a), _p(self.ipiv), _p(y))
        return y


def fem_interpolate(M, L, d, X, Y):
    d = _f64(d)
    X = np.atleast_1d(np.asarray(X, np.float64))
    Y = np.atleast_1d(np.asarray(Y, np.float64))
    out = np.empty(X.shape)
    f = lib().orc_fem_interpolate
    for t in range(X.size):
        out.flat[t] = f(M, float(L), _p(d), float(X.flat[t]), float(Y.flat[t]))
    return out


def fine_to_coarse(N, solid, u, px, py):
    u = _f64(u)
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    px = np.atleast_1d(np.asarray(px, np.float64))
    py = np.atleast_1d(np.asarray(py, np.float64))
    out = np.empty(px.shape)
    f = lib().orc_fine_to_coarse
    for t in range(px.size):
        out.flat[t] = f(N, _p(solid), _p(u), float(px.flat[t]), float(py.flat[t]))
    return out


from .hybrid import HybridOracle, coarse_dirichlet_sets, run_hybrid  # noqa: E402,F401
