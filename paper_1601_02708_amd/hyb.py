"""Python binding of the C ABI in include/hyb.h (ctypes; marshalling only).

Every step of the method runs in libhyb.so's HIP kernels.  PyTorch only
supplies device memory (the three population buffers and the workspace)
and the stream.  Importing this module does not need a GPU; creating a
``Hybrid`` does, and fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhyb.so")

HYB_OK, HYB_EINVAL, HYB_EHIP, HYB_ENOCONV, HYB_ENONFINITE = 0, -1, -2, -3, -4
HYB_FP64, HYB_FP32, HYB_FP16S = 0, 1, 2
PRECISIONS = {"fp64": HYB_FP64, "fp32": HYB_FP32, "fp16s": HYB_FP16S}
HYB_F2C, HYB_C2F = 0, 1
HYB_FINE, HYB_COARSE = 0, 1
HYB_BC_DIRICHLET, HYB_BC_NEUMANN = 0, 1
HYB_OVERLAP_AUTO = -1

_P = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


class HybMesh(ctypes.Structure):
    _fields_ = [("M", _i), ("L", _d), ("outer_value", _d), ("overlap_elems", _i), ("supg", _i), ("d0", _P),
                ("outer_natural", _i)]


class HybLattice(ctypes.Structure):
    _fields_ = [("N", _i), ("x0", _d), ("y0", _d), ("precision", _i), ("tau", _d), ("eta", _i),
                ("bc_clamp", _i), ("solid", _P), ("u0", _P), ("f_buf", _P * 3), ("workspace", _P),
                ("stream", _P), ("dissolution", _i), ("wall_closure", _i)]


class HybVelocity(ctypes.Structure):
    _fields_ = [("fine", _P), ("coarse", _P)]


class HybReaction(ctypes.Structure):
    _fields_ = [("k", _d), ("k_field", _P)]


class HybRunStats(ctypes.Structure):
    _fields_ = [("infeasible", ctypes.c_int64), ("nonfinite", ctypes.c_int64), ("krylov_iters", ctypes.c_int32),
                ("krylov_converged", ctypes.c_int32), ("krylov_relres", _d), ("coarse_steps", ctypes.c_int64),
                ("fine_steps", ctypes.c_int64), ("overlap_depth", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("mass", ctypes.c_double), ("min_f", ctypes.c_double), ("h_function", ctypes.c_double)]


class Hyb1DParams(ctypes.Structure):
    _fields_ = [("h_c", _d), ("h_f", _d), ("L_ov", _d), ("max_iter", _i), ("v", _d), ("D", _d)]


# exported symbol -> (restype, argtypes); mirrors include/hyb.h and include/hyb1d.h
SIGNATURES = {
    "hyb_query": (_i, [_P, _P, _P, _P]),
    "hyb_create": (_i, [_P, _P, _d, _P, _P, _P]),
    "hyb_interface_exchange": (_i, [_P, _i]),
    "hyb_coarse_step": (_i, [_P, _i]),
    "hyb_lbm_substeps": (_i, [_P, _i, _i]),
    "hyb_commit": (_i, [_P]),
    "hyb_step": (_i, [_P, _i]),
    "hyb_set_boundary": (_i, [_P, _P, _P, _P]),
    "hyb_concentration": (_i, [_P, _i, _P, _i]),
    "hyb_get_populations": (_i, [_P, _P]),
    "hyb_populations_device": (_i, [_P, _P]),
    "hyb_set_populations": (_i, [_P, _P]),
    "hyb_stats": (_i, [_P, _P]),
    "hyb_set_wall_normals": (_i, [_P, _P]),
    "hyb_diagnostics": (_i, [_P, _P, _i]),
    "hyb_diagnostics_noalloc": (_i, [_P, _P]),
    "hyb_layout": (_i, [_P, _P, _P]),
    "hyb_adjoint_query": (_i, [_P, _i, _P]),
    "hyb_lbm_substeps_record": (_i, [_P, _i, _P]),
    "hyb_lbm_adjoint": (_i, [_P, _i, _P, _P, _P, _P, _P, _P]),
    "hyb_step_adjoint_query": (_i, [_P, _i, _P]),
    "hyb_step_record": (_i, [_P, _i, _P]),
    "hyb_step_adjoint": (_i, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "hyb_set_coarse": (_i, [_P, _P]),
    "hyb_set_reaction_field": (_i, [_P, _P]),
    "hyb_set_outer_value": (_i, [_P, _d]),
    "hyb_set_dissolution": (_i, [_P, _d, _d, _P]),
    "hyb_dissolution_state": (_i, [_P, _P, _P, _P]),
    "hyb_set_solids": (_i, [_P, _P, _P]),
    "hyb_checkpoint_query": (_i, [_P, _P]),
    "hyb_checkpoint_save": (_i, [_P, _P]),
    "hyb_checkpoint_load": (_i, [_P, _P]),
    "hyb_set_overlap": (_i, [_P, _i]),
    "hyb_set_steps_per_launch": (_i, [_P, _i]),
    "hyb_kernel_timing": (_i, [_P, _i]),
    "hyb_kernel_time": (_i, [_P, _P, _P]),
    "hyb_destroy": (None, [_P]),
    "hyb_group_query": (_i, [_P, _i, _P, _P]),
    "hyb_group_create": (_i, [_P, _i, _P, _d, _P, _d, _P, _P, _P]),
    "hyb_group_step": (_i, [_P, _i]),
    "hyb_group_coarse": (_i, [_P, _P, _i]),
    "hyb_group_destroy": (None, [_P]),
    "hyb_group_last_error": (ctypes.c_char_p, [_P]),
    "hyb1d_query": (_i, [_P, _P, _P, _P, _P, _P]),
    "hyb1d_create": (_i, [_P, _P, _P, _P, _P, _P]),
    "hyb1d_run": (_i, [_P, _i]),
    "hyb1d_state": (_i, [_P, _P, _P]),
    "hyb1d_destroy": (None, [_P]),
    "hyb_last_error": (ctypes.c_char_p, [_P]),
}

_LIB = None

# Handles still open, closed by an exit hook before the interpreter and the
# HIP runtime are torn down: a handle owns a HIP stream and events, and
# destroying them after the runtime (or a profiler attached to it) has shut
# down faults the process on its way out.  Groups close before the patch
# handles they couple.
_LIVE_GROUPS = weakref.WeakSet()
_LIVE_HANDLES = weakref.WeakSet()
_EXIT_HOOK = False


def _close_live():
    for objs in (_LIVE_GROUPS, _LIVE_HANDLES):
        for o in list(objs):
            try:
                o.close()
            except Exception:
                pass


def _track(obj, group=False):
    global _EXIT_HOOK
    if not _EXIT_HOOK:
        # registered after torch's own hooks (torch is imported first), so it
        # runs before them: Python runs exit hooks last-registered first
        import torch  # noqa: F401
        atexit.register(_close_live)
        _EXIT_HOOK = True
    (_LIVE_GROUPS if group else _LIVE_HANDLES).add(obj)


class HybError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hyb error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhyb.so (no GPU needed to load).  Raises if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data


class Hybrid:
    """One simulation handle: the fine lattice patch and (optionally) the
    coarse mesh around it.  Arrays follow include/hyb.h."""

    def __init__(self, *, N, x0, y0, u0, vx, vy, D, eta, precision="fp64", tau=0.0, solid=None,
                 k=0.0, k_field=None, bc_clamp=0, mesh=None, device=None, dissolution=False, wall_closure=False):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("Hybrid needs a GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.dev = torch.device(device or "cuda:0")
        self.N, self.eta = int(N), int(eta)
        self.precision = precision
        self._keep = []

        def host(a, dt):
            arr = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(arr)
            return arr

        u0h = host(np.asarray(u0).reshape(N, N), np.float64)
        vel = host(np.stack([np.asarray(vx).reshape(N, N), np.asarray(vy).reshape(N, N)]), np.float32)
        solidh = None if solid is None else host(np.asarray(solid).reshape(N, N), np.uint8)
        kfh = None if k_field is None else host(np.asarray(k_field).reshape(N, N), np.float64)

        self.lat = HybLattice()
        self.lat.N = self.N
        self.lat.x0, self.lat.y0 = float(x0), float(y0)
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.lat.precision = PRECISIONS[precision]
        self.lat.tau = float(tau)
        self.lat.eta = self.eta
        self.lat.bc_clamp = int(bc_clamp)
        self.lat.solid = _ptr(solidh)
        self.lat.u0 = _ptr(u0h)
        self.lat.dissolution = int(bool(dissolution))
        self.lat.wall_closure = int(bool(wall_closure))
        self.dissolution = bool(dissolution)
        self.meshs = None
        vc = None
        if mesh is not None:
            self.M = int(mesh["M"])
            d0 = host(np.asarray(mesh["d0"]).ravel(), np.float64)
            vc = host(np.asarray(mesh["v"]).reshape(-1, 2), np.float64)
            self.meshs = HybMesh(self.M, float(mesh["L"]), float(mesh.get("outer_value", 0.0)),
                                 int(mesh.get("overlap_elems", 1)), int(mesh.get("supg", 1)), _ptr(d0),
                                 int(mesh.get("outer_natural", 0)))
        else:
            self.M = 0
        fb = ctypes.c_size_t()
        wb = ctypes.c_size_t()
        mp = ctypes.addressof(self.meshs) if self.meshs is not None else None
        rc = lib.hyb_query(mp, ctypes.addressof(self.lat), ctypes.addressof(fb), ctypes.addressof(wb))
        if rc != HYB_OK:
            raise HybError(rc, "hyb_query rejected the problem")
        self.f_bytes, self.ws_bytes = fb.value, wb.value
        self.fbuf = [torch.empty(self.f_bytes, dtype=torch.uint8, device=self.dev) for _ in range(3)]
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.dev)
        for b in range(3):
            self.lat.f_buf[b] = self.fbuf[b].data_ptr()
        self.lat.workspace = self.ws.data_ptr()
        self.stream = torch.cuda.current_stream(self.dev)
        self.lat.stream = self.stream.cuda_stream
        self.vel = HybVelocity(_ptr(vel), _ptr(vc))
        self.react = HybReaction(float(k), _ptr(kfh))
        h = ctypes.c_void_p()
        rc = lib.hyb_create(mp, ctypes.addressof(self.lat), float(D), ctypes.addressof(self.vel),
                            ctypes.addressof(self.react), ctypes.addressof(h))
        if rc != HYB_OK:
            raise HybError(rc, "hyb_create failed (see stderr)")
        self.h = h
        _track(self)
        self._keep.clear()

    @classmethod
    def from_problem(cls, problem, precision="fp64", tau=None, mesh=True, **kw):
        cfg = problem.cfg
        m = None
        if mesh:
            m = dict(M=cfg.M, L=problem.L, outer_value=kw.pop("outer_value", cfg.outer_value),
                     overlap_elems=cfg.overlap_elems, supg=cfg.supg, d0=problem.u0_coarse, v=problem.vc,
                     outer_natural=kw.pop("outer_natural", cfg.outer_natural))
        return cls(N=cfg.N, x0=problem.x0, y0=problem.y0, u0=problem.u0_fine, vx=problem.vx, vy=problem.vy,
                   D=cfg.D, eta=kw.pop("eta", cfg.eta), precision=precision,
                   tau=(cfg.tau or 0.0) if tau is None else tau, solid=problem.solid, k=cfg.k,
                   k_field=kw.pop("k_field", problem.k_field),
                   bc_clamp=cfg.bc_clamp, mesh=m, **kw)

    # -- calls ------------------------------------------------------------
    def _check(self, rc):
        if rc != HYB_OK:
            raise HybError(rc, load().hyb_last_error(self.h).decode())
        return rc

    def interface_exchange(self, direction):
        return self._check(load().hyb_interface_exchange(self.h, direction))

    def coarse_step(self, max_iter=0):
        return self._check(load().hyb_coarse_step(self.h, max_iter))

    def lbm_substeps(self, n_sub, restart=1):
        return self._check(load().hyb_lbm_substeps(self.h, n_sub, restart))

    def commit(self):
        return self._check(load().hyb_commit(self.h))

    def step(self, max_schwarz):
        return self._check(load().hyb_step(self.h, max_schwarz))

    def set_boundary(self, a, b=None, kind=None):
        P = 4 * (self.N - 1)
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (P,)))
        b = None if b is None else np.ascontiguousarray(np.broadcast_to(np.asarray(b, np.float64), (P,)))
        kind = None if kind is None else np.ascontiguousarray(kind, np.int8)
        return self._check(load().hyb_set_boundary(self.h, _ptr(kind), _ptr(a), _ptr(b)))

    def concentration(self, which=HYB_FINE):
        n = self.N * self.N if which == HYB_FINE else (self.M + 1) ** 2
        out = np.empty(n)
        self._check(load().hyb_concentration(self.h, which, out.ctypes.data, 0))
        return out.reshape(self.N, self.N) if which == HYB_FINE else out

    def concentration_device(self, out_tensor, which=HYB_FINE):
        return self._check(load().hyb_concentration(self.h, which, out_tensor.data_ptr(), 1))

    def get_populations(self):
        out = np.empty((9, self.N, self.N))
        self._check(load().hyb_get_populations(self.h, out.ctypes.data))
        return out

    def populations_device(self, out_tensor):
        """Current fine state into a device FP64 tensor [9, N, N] (stream-ordered)."""
        return self._check(load().hyb_populations_device(self.h, out_tensor.data_ptr()))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64)
        return self._check(load().hyb_set_populations(self.h, f.ctypes.data))

    def stats(self):
        s = HybRunStats()
        self._check(load().hyb_stats(self.h, ctypes.addressof(s)))
        return {k: getattr(s, k) for k, _ in HybRunStats._fields_}

    def diagnostics(self, out=None):
        """(mass, min f*, H, non-finite nodes) of the current fine state.
        With ``out`` (a CUDA float64 tensor of >= 4 elements) the values are
        written there on the handle's stream and nothing is returned."""
        if out is not None:
            if out.device.type != "cuda" or out.dtype != self.torch.float64 or out.numel() < 4:
                raise ValueError("out must be a CUDA float64 tensor of at least 4 elements")
            self._check(load().hyb_diagnostics(self.h, out.data_ptr(), 1))
            return None
        v = np.zeros(4)
        self._check(load().hyb_diagnostics(self.h, v.ctypes.data, 0))
        return {"mass": float(v[0]), "min_f": float(v[1]), "h_function": float(v[2]), "nonfinite": int(v[3])}

    # -- reverse mode of a whole coarse step ---------------------------------
    def step_tape(self, passes):
        """A device tape (torch uint8 tensor) for hyb_step_record(passes)."""
        nb = ctypes.c_size_t()
        self._check(load().hyb_step_adjoint_query(self.h, int(passes), ctypes.addressof(nb)))
        return self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.dev)

    def step_record(self, passes, tape):
        return self._check(load().hyb_step_record(self.h, int(passes), tape.data_ptr()))

    def step_adjoint(self, tape, lam_f, lam_d, lam_f_out, lam_d_out, grad_k=None, grad_outer=None, lam_sub=None):
        """Device FP64 tensors: lam_f/lam_f_out [9, N, N], lam_d/lam_d_out
        [(M+1)^2] (lam_d may be None), grad_k [N, N] and grad_outer
        [(M+1)^2] or None (added to); lam_sub [9, N, N] or None: the
        cotangent of every intermediate fine state of the committed pass."""
        t = self.torch
        for x in (lam_f, lam_f_out, lam_d_out) + tuple(v for v in (lam_d, grad_k, grad_outer, lam_sub)
                                                         if v is not None):
            if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous():
                raise ValueError("adjoint arrays must be contiguous FP64 device tensors")
        ptr = lambda v: None if v is None else v.data_ptr()
        return self._check(load().hyb_step_adjoint(self.h, tape.data_ptr(), lam_f.data_ptr(), ptr(lam_sub),
                                                   ptr(lam_d), lam_f_out.data_ptr(), lam_d_out.data_ptr(),
                                                   ptr(grad_k), ptr(grad_outer)))

    def step_reading_substeps(self, passes, read):
        """One coarse step of Algorithm 1 through the separate calls
        (transfers, coarse solve, fine steps, commit) so that ``read()`` can
        look at every intermediate fine state f*(t_n + j), j = 1 .. eta-1, of
        the committed (last) pass; the step's result equals hyb_step's (in
        FP64 bit for bit: the same per-node operations, single-step
        launches).  A coarse solve that ran out of its launch budget repeats
        the step from the untouched committed state; ``read`` returns a value
        for each state and the values of the attempt that committed are
        returned."""
        lib = load()
        for attempt in range(20):
            vals = []
            self.lbm_substeps(0, restart=1)          # the fine state read first is the committed one
            for it in range(passes):
                self.interface_exchange(HYB_F2C)
                self.coarse_step(200)
                self.interface_exchange(HYB_C2F)
                if it < passes - 1:
                    self.lbm_substeps(self.eta, restart=1)
                    continue
                for j in range(1, self.eta + 1):
                    self.lbm_substeps(1, restart=1 if j == 1 else 0)
                    if j < self.eta:
                        vals.append(read())
            rc = lib.hyb_commit(self.h)
            if rc == HYB_OK:
                return vals
            if rc != HYB_ENOCONV:
                self._check(rc)
        raise HybError(HYB_ENOCONV, "coarse solve did not converge in 20 attempts")

    def set_coarse(self, d):
        """Replace the committed coarse solution (host [(M+1)^2] FP64)."""
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1)
        if d.size != (self.M + 1) ** 2:
            raise ValueError("coarse state must have (M+1)^2 entries")
        return self._check(load().hyb_set_coarse(self.h, _ptr(d)))

    def set_reaction_field(self, k_field):
        """Replace the fine per-node reaction rate (host [N, N], values in [0, 1))."""
        k = np.ascontiguousarray(k_field, dtype=np.float64).reshape(-1)
        if k.size != self.N * self.N:
            raise ValueError("k_field must have N*N entries")
        return self._check(load().hyb_set_reaction_field(self.h, _ptr(k)))

    def set_outer_value(self, value):
        """Replace the Dirichlet value of the outer edges that are not natural."""
        return self._check(load().hyb_set_outer_value(self.h, float(value)))

    # -- device checkpoints ---------------------------------------------------
    def checkpoint(self):
        """A device checkpoint (torch uint8 tensor) of the committed state."""
        nb = ctypes.c_size_t()
        self._check(load().hyb_checkpoint_query(self.h, ctypes.addressof(nb)))
        t = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.dev)
        self._check(load().hyb_checkpoint_save(self.h, t.data_ptr()))
        return t

    def restore(self, ckpt):
        """Return to a state saved by checkpoint()."""
        return self._check(load().hyb_checkpoint_load(self.h, ckpt.data_ptr()))

    # -- dissolving solids ---------------------------------------------------
    def set_wall_normals(self, normals):
        """Maximum-entropy zero-flux closure at solid walls with the given
        unit outward normals (host [2, N, N], pointing into the solid), or
        bounce-back again with None (handle created with wall_closure=True)."""
        if normals is None:
            return self._check(load().hyb_set_wall_normals(self.h, None))
        n = np.ascontiguousarray(normals, dtype=np.float32).reshape(-1)
        if n.size != 2 * self.N * self.N:
            raise ValueError("normals must have 2*N*N entries")
        return self._check(load().hyb_set_wall_normals(self.h, n.ctypes.data))

    def set_dissolution(self, kappa_s, c_sat, mass=None):
        """Surface reaction rate and saturation concentration at fluid-solid
        links, and the solid masses (host [N, N], read at solid nodes)."""
        m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
        if m is not None and m.size != self.N * self.N:
            raise ValueError("mass must have N*N entries")
        return self._check(load().hyb_set_dissolution(self.h, float(kappa_s), float(c_sat), _ptr(m)))

    def set_solids(self, solid, mass):
        """Replace the geometry (host [N, N] flags, only nodes solid at
        creation) and the masses (host [N, N])."""
        sol = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        m = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
        if sol.size != self.N * self.N or m.size != self.N * self.N:
            raise ValueError("solid and mass must have N*N entries")
        return self._check(load().hyb_set_solids(self.h, _ptr(sol), _ptr(m)))

    def dissolution_state(self):
        """(solid flags [N, N] uint8, masses [N, N], solids converted so far)."""
        sol = np.empty((self.N, self.N), np.uint8)
        mass = np.empty((self.N, self.N), np.float64)
        conv = ctypes.c_int64()
        self._check(load().hyb_dissolution_state(self.h, _ptr(sol), _ptr(mass), ctypes.addressof(conv)))
        return sol, mass, conv.value

    # -- reverse mode -------------------------------------------------------
    def adjoint_tape(self, n_sub):
        """A device tape (torch uint8 tensor) for n_sub recorded fine steps."""
        nb = ctypes.c_size_t()
        self._check(load().hyb_adjoint_query(self.h, int(n_sub), ctypes.addressof(nb)))
        return self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.dev)

    def substeps_record(self, n_sub, tape):
        return self._check(load().hyb_lbm_substeps_record(self.h, int(n_sub), tape.data_ptr()))

    def adjoint(self, n_sub, tape, lam_in, lam_out, grad_a, grad_b, grad_k=None):
        """Device FP64 tensors: lam_in/lam_out [9, N, N], grad_a/grad_b [4(N-1)],
        grad_k [N, N] or None (gradients are added to)."""
        t = self.torch
        for x in (lam_in, lam_out, grad_a, grad_b) + (() if grad_k is None else (grad_k,)):
            if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous():
                raise ValueError("adjoint arrays must be contiguous FP64 device tensors")
        return self._check(load().hyb_lbm_adjoint(self.h, int(n_sub), tape.data_ptr(), lam_in.data_ptr(),
                                                  lam_out.data_ptr(), grad_a.data_ptr(), grad_b.data_ptr(),
                                                  None if grad_k is None else grad_k.data_ptr()))

    def set_overlap(self, depth):
        """Deep interior tiles of the first `depth` multi-step launches of each
        Schwarz pass overlap the pass's coarse work (0: serial order;
        HYB_OVERLAP_AUTO: the next steps tune the depth)."""
        return self._check(load().hyb_set_overlap(self.h, int(depth)))

    def set_steps_per_launch(self, steps):
        """Most fine steps per sweep launch, 1 to 5 (default 5 fp32, 4 fp64, 4 fp16s);
        2 or more also reverses the adjoint's fine steps in pairs."""
        return self._check(load().hyb_set_steps_per_launch(self.h, int(steps)))

    def kernel_timing(self, enable=True):
        return self._check(load().hyb_kernel_timing(self.h, int(enable)))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(load().hyb_kernel_time(self.h, ctypes.addressof(ms), ctypes.addressof(n)))
        return ms.value, n.value

    def layout(self):
        p = ctypes.c_size_t()
        q = ctypes.c_size_t()
        self._check(load().hyb_layout(self.h, ctypes.addressof(p), ctypes.addressof(q)))
        return p.value, q.value

    def close(self):
        if getattr(self, "h", None):
            load().hyb_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has closed every live handle;
        # never call into the HIP runtime from a finaliser then (the check is
        # bound here: module globals such as sys may already be None)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def lattice_substeps_function():
    """torch.autograd.Function for f*(n_sub) = F(f*(0), a, b) on a handle:
    forward records the fine steps, backward runs the C ABI adjoint.  Usage:
    ``LatticeSubsteps = lattice_substeps_function()`` then
    ``LatticeSubsteps.apply(hybrid, n_sub, f0, a, b)`` with f0 [9, N, N] and
    a, b [4(N-1)] FP64 tensors; returns f*(n_sub) [9, N, N] on f0's device."""
    import torch

    class LatticeSubsteps(torch.autograd.Function):
        @staticmethod
        def forward(ctx, g, n_sub, f0, a, b):
            g.set_populations(f0.detach().cpu().numpy())
            g.set_boundary(a.detach().cpu().numpy(), b.detach().cpu().numpy())
            tape = g.adjoint_tape(n_sub)
            g.substeps_record(n_sub, tape)
            out = torch.from_numpy(g.get_populations()).to(f0.device)
            ctx.g, ctx.n_sub, ctx.tape = g, n_sub, tape
            ctx.dev = f0.device
            return out

        @staticmethod
        def backward(ctx, grad_out):
            g = ctx.g
            lam = grad_out.detach().to(device=g.dev, dtype=torch.float64).contiguous()
            lam_out = torch.empty_like(lam)
            P = 4 * (g.N - 1)
            ga = torch.zeros(P, dtype=torch.float64, device=g.dev)
            gb = torch.zeros(P, dtype=torch.float64, device=g.dev)
            g.adjoint(ctx.n_sub, ctx.tape, lam, lam_out, ga, gb)
            return None, None, lam_out.to(ctx.dev), ga.to(ctx.dev), gb.to(ctx.dev)

    return LatticeSubsteps



def steps_adjoint(g, n_steps, cotangent, passes, checkpoint_every=8, state_in_cotangent=True, substep_weight=None):
    """Reverse mode of n_steps coarse steps from the handle's committed state
    (which is left at the end of the rollout), with the committed state
    checkpointed on the device every ``checkpoint_every`` steps
    (hyb_checkpoint_save: populations, coarse state and, with dissolving
    solids, geometry and masses) and each segment re-run from its
    checkpoint, so every step runs twice forwards and once backwards.

    ``cotangent(n, F, d)`` returns (dJ/dF_n, dJ/dd_n) as host FP64 arrays or
    device tensors ([9, N, N], [(M+1)^2]; either may be None; a device FP64
    tensor is added without a copy) for the state (F, d) after
    step n (n = 1 .. n_steps), so J may sum over the whole trajectory; with
    ``state_in_cotangent`` False it receives None for F and d (no host copy
    of the state is made).  Every step runs ``passes`` Schwarz passes
    (hyb_step with that count).  Returns host FP64 arrays (dJ/dF_0, dJ/dd_0,
    dJ/dk, dJ/dg_outer): the initial state, the fine per-node reaction rate
    and the outer-edge Dirichlet values (per coarse node, summed over the
    steps).  ``substep_weight`` ([9, N, N] host array or device tensor, or
    None): J also holds <w, f*(t)> for every intermediate fine state of
    every step's committed pass (so, with the same w in ``cotangent``, J can
    sum over every fine step).  Each step's adjoint runs on the GPU through
    hyb_step_record and hyb_step_adjoint; this function only orchestrates."""
    import torch
    N, M = g.N, g.M
    dev = g.dev
    n1 = (M + 1) ** 2
    lam_sub = None
    if substep_weight is not None:
        lam_sub = (substep_weight.to(device=dev, dtype=torch.float64).contiguous() if torch.is_tensor(substep_weight)
                   else torch.from_numpy(np.ascontiguousarray(substep_weight, np.float64)).to(dev))

    # forward rollout, checkpointing the state at every segment start
    ckpt = {}
    for n in range(n_steps):
        if n % checkpoint_every == 0:
            ckpt[n] = g.checkpoint()
        g.step(passes)
    ckpt[n_steps] = g.checkpoint()
    tape = g.step_tape(passes)
    lam_f = torch.zeros((9, N, N), dtype=torch.float64, device=dev)
    lam_d = torch.zeros(n1, dtype=torch.float64, device=dev)
    out_f = torch.empty_like(lam_f)
    out_d = torch.empty_like(lam_d)
    gk = torch.zeros((N, N), dtype=torch.float64, device=dev)
    gouter = torch.zeros(n1, dtype=torch.float64, device=dev)
    starts = sorted(k for k in ckpt if k < n_steps)
    for si in range(len(starts) - 1, -1, -1):
        s0 = starts[si]
        s1 = starts[si + 1] if si + 1 < len(starts) else n_steps
        # re-run the segment: seg[i] is the state before step s0 + i
        g.restore(ckpt[s0])
        seg = [ckpt[s0]]
        for _ in range(s0, s1 - 1):
            g.step(passes)
            seg.append(g.checkpoint())
        for n in range(s1 - 1, s0 - 1, -1):
            g.restore(seg[n - s0])
            g.step_record(passes, tape)
            # the handle now holds the state after step n
            if state_in_cotangent:
                cf, cd = cotangent(n + 1, g.get_populations(), g.concentration(HYB_COARSE).copy())
            else:
                cf, cd = cotangent(n + 1, None, None)
            if cf is not None:
                lam_f += (cf.to(device=dev, dtype=torch.float64) if torch.is_tensor(cf)
                          else torch.from_numpy(np.ascontiguousarray(cf, np.float64)).to(dev))
            if cd is not None:
                lam_d += (cd.to(device=dev, dtype=torch.float64).reshape(-1) if torch.is_tensor(cd)
                          else torch.from_numpy(np.ascontiguousarray(cd, np.float64).reshape(-1)).to(dev))
            g.step_adjoint(tape, lam_f, lam_d, out_f, out_d, gk, gouter, lam_sub)
            lam_f, out_f = out_f, lam_f
            lam_d, out_d = out_d, lam_d
        del seg
    g.restore(ckpt[n_steps])
    return lam_f.cpu().numpy(), lam_d.cpu().numpy(), gk.cpu().numpy(), gouter.cpu().numpy()


def trajectory_functional(every_substep=False):
    """torch.autograd.Function for a linear functional summed over a
    trajectory of coarse steps,

        J(k, g) = sum_{n=1}^{n_steps} <w_f, F_n> + <w_d, d_n>,

    or, with ``every_substep``, over every fine step,

        J(k, g) = sum_{n} [ sum_{j=1}^{eta} <w_f, f*(t_{n-1} + j)> + <w_d, d_n> ]

    (the fine states of each step's committed Schwarz pass; the forward then
    runs each step through the separate calls, Hybrid.step_reading_substeps,
    and the backward injects w_f at every reversed fine state),

    as a function of the fine per-node reaction rate k and the Dirichlet
    value g of the outer edges that are not natural, from the handle's
    committed state at the call (the outlet flux of a patch edge is such a
    functional: w_f = e_x on the edge nodes).  ``Functional =
    trajectory_functional()`` then ``Functional.apply(hybrid, n_steps,
    passes, checkpoint_every, w_f, w_d, k, g)`` with w_f host [9, N, N] (or
    None), w_d host [(M+1)^2] (or None), k an FP64 tensor [N, N] and g a 0-d
    FP64 tensor.  Forward sets the controls on the handle
    (hyb_set_reaction_field, hyb_set_outer_value), runs the steps and
    accumulates J on the device; backward returns to the start state and runs
    steps_adjoint (checkpoints every ``checkpoint_every`` steps, every step's
    adjoint on the GPU).  dJ/dk and dJ/dg are partial derivatives at a fixed
    start state; the handle is left at the end of the rollout."""
    import torch

    class Functional(torch.autograd.Function):
        @staticmethod
        def forward(ctx, g, n_steps, passes, checkpoint_every, w_f, w_d, k, gval):
            N, n1 = g.N, (g.M + 1) ** 2
            dev = g.dev
            kh = k.detach().to("cpu", torch.float64).numpy()
            gv = float(gval)
            ctx.start = g.checkpoint()
            g.set_reaction_field(kh)
            g.set_outer_value(gv)
            J = torch.zeros((), dtype=torch.float64, device=dev)
            wf = None if w_f is None else torch.from_numpy(np.ascontiguousarray(w_f, np.float64)).to(dev)
            wd = None if w_d is None else torch.from_numpy(
                np.ascontiguousarray(w_d, np.float64).reshape(-1)).to(dev)
            fbuf = torch.empty((9, N, N), dtype=torch.float64, device=dev) if wf is not None else None
            dbuf = torch.empty(n1, dtype=torch.float64, device=dev) if wd is not None else None
            def read():
                g.populations_device(fbuf)
                return (fbuf * wf).sum()

            for _ in range(n_steps):
                if every_substep and wf is not None:
                    for v in g.step_reading_substeps(passes, read):
                        J += v
                else:
                    g.step(passes)
                if wf is not None:
                    g.populations_device(fbuf)
                    J += (fbuf * wf).sum()
                if wd is not None:
                    g.concentration_device(dbuf, HYB_COARSE)
                    J += (dbuf * wd).sum()
            ctx.g, ctx.n_steps, ctx.passes, ctx.every = g, n_steps, passes, checkpoint_every
            ctx.w = (w_f, w_d)
            ctx.controls = (kh, gv)
            ctx.k_meta = (k.dtype, k.device)
            ctx.g_meta = (gval.dtype, gval.device) if torch.is_tensor(gval) else None
            return J

        @staticmethod
        def backward(ctx, gJ):
            g = ctx.g
            g.restore(ctx.start)
            g.set_reaction_field(ctx.controls[0])
            g.set_outer_value(ctx.controls[1])
            w_f, w_d = ctx.w
            dev = g.dev
            # the weights go to the device once; every step adds the same tensors
            wf = None if w_f is None else torch.from_numpy(np.ascontiguousarray(w_f, np.float64)).to(dev)
            wd = None if w_d is None else torch.from_numpy(
                np.ascontiguousarray(w_d, np.float64).reshape(-1)).to(dev)
            _, _, gk, go = steps_adjoint(g, ctx.n_steps, lambda n, F, d: (wf, wd), ctx.passes,
                                         checkpoint_every=ctx.every, state_in_cotangent=False,
                                         substep_weight=wf if every_substep else None)
            dt, dv = ctx.k_meta
            grad_k = torch.from_numpy(gk).to(device=dv, dtype=dt) * gJ.to(dv)
            grad_g = None
            if ctx.g_meta is not None:
                grad_g = (gJ * float(go.sum())).to(device=ctx.g_meta[1], dtype=ctx.g_meta[0])
            return None, None, None, None, None, None, grad_k, grad_g

    return Functional


def rollout_function():
    """torch.autograd.Function for (F_n, d_n) = n coarse steps of Algorithm 1
    from (F_0, d_0) on a handle: ``Rollout = rollout_function()`` then
    ``Rollout.apply(hybrid, n_steps, passes, F0, d0)`` with F0 [9, N, N] and
    d0 [(M+1)^2] FP64 tensors; backward runs steps_adjoint (checkpointed,
    every step's adjoint on the GPU)."""
    import torch

    class Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, g, n_steps, passes, F0, d0):
            # with dissolving solids the rollout starts from the handle's
            # current geometry, which backward restores
            ctx.geom = g.dissolution_state()[:2] if getattr(g, "dissolution", False) else None
            g.set_populations(F0.detach().cpu().numpy())
            g.set_coarse(d0.detach().cpu().numpy())
            for _ in range(n_steps):
                g.step(passes)
            ctx.g, ctx.n, ctx.passes, ctx.dev = g, n_steps, passes, F0.device
            ctx.F0, ctx.d0 = F0.detach().cpu().numpy(), d0.detach().cpu().numpy()
            return (torch.from_numpy(g.get_populations()).to(F0.device),
                    torch.from_numpy(g.concentration(HYB_COARSE).copy()).to(F0.device))

        @staticmethod
        def backward(ctx, gF, gd):
            g, n = ctx.g, ctx.n
            end = (g.get_populations(), g.concentration(HYB_COARSE).copy())
            end_geom = g.dissolution_state()[:2] if ctx.geom is not None else None
            if ctx.geom is not None:
                g.set_solids(*ctx.geom)
            g.set_populations(ctx.F0)
            g.set_coarse(ctx.d0)
            cF = None if gF is None else gF.detach().cpu().numpy()
            cd = None if gd is None else gd.detach().cpu().numpy()
            lF, ld, _, _ = steps_adjoint(g, n, lambda k, F, d: (cF, cd) if k == n else (None, None),
                                         ctx.passes, checkpoint_every=max(1, n))
            if end_geom is not None:
                g.set_solids(*end_geom)
            g.set_populations(end[0])
            g.set_coarse(end[1])
            return None, None, None, torch.from_numpy(lF).to(ctx.dev), torch.from_numpy(ld).to(ctx.dev)

    return Rollout


# ----------------------------------------------------------------------------
# several fine patches around one coarse subdomain (Algorithm 2)
# ----------------------------------------------------------------------------

class HybridGroup:
    """Lattice-only Hybrid patches (created with mesh=None) coupled through
    one coarse mesh: ``mesh`` as for Hybrid (M, L, outer_value,
    overlap_elems, supg, d0, v), D and the uniform coarse rate k."""

    def __init__(self, patches, mesh, D, k=0.0):
        lib = load()
        self.patches = list(patches)
        p0 = self.patches[0]
        self.torch, self.dev, self.stream = p0.torch, p0.dev, p0.stream
        self.M = int(mesh["M"])
        d0 = np.ascontiguousarray(np.asarray(mesh["d0"]).ravel(), np.float64)
        vc = np.ascontiguousarray(np.asarray(mesh["v"]).reshape(-1, 2), np.float64)
        self._keep = [d0, vc]
        self.meshs = HybMesh(self.M, float(mesh["L"]), float(mesh.get("outer_value", 0.0)),
                             int(mesh.get("overlap_elems", 1)), int(mesh.get("supg", 1)), _ptr(d0),
                             int(mesh.get("outer_natural", 0)))
        lats = (HybLattice * len(self.patches))()
        for i, p in enumerate(self.patches):
            lats[i] = p.lat
        wb = ctypes.c_size_t()
        rc = lib.hyb_group_query(ctypes.addressof(self.meshs), len(self.patches), ctypes.addressof(lats),
                                 ctypes.addressof(wb))
        if rc != HYB_OK:
            raise HybError(rc, "hyb_group_query rejected the set-up")
        self.ws = self.torch.empty(wb.value, dtype=self.torch.uint8, device=self.dev)
        hs = (ctypes.c_void_p * len(self.patches))(*[p.h.value for p in self.patches])
        g = ctypes.c_void_p()
        rc = lib.hyb_group_create(ctypes.addressof(self.meshs), len(self.patches), ctypes.addressof(hs), float(D),
                                  _ptr(vc), float(k), self.ws.data_ptr(), self.stream.cuda_stream, ctypes.addressof(g))
        if rc != HYB_OK:
            raise HybError(rc, "hyb_group_create failed (see stderr)")
        self.g = g
        _track(self, group=True)

    def step(self, max_schwarz):
        rc = load().hyb_group_step(self.g, int(max_schwarz))
        if rc != HYB_OK:
            raise HybError(rc, load().hyb_group_last_error(self.g).decode())

    def coarse(self):
        out = np.empty((self.M + 1, self.M + 1))
        rc = load().hyb_group_coarse(self.g, _ptr(out), 0)
        if rc != HYB_OK:
            raise HybError(rc, load().hyb_group_last_error(self.g).decode())
        return out

    def close(self):
        if getattr(self, "g", None):
            load().hyb_group_destroy(self.g)
            self.g = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has closed every live handle;
        # never call into the HIP runtime from a finaliser then (the check is
        # bound here: module globals such as sys may already be None)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# one-dimensional hybrid (include/hyb1d.h)
# ----------------------------------------------------------------------------

def hybrid1d_sizes(h_c, h_f, L_ov, max_iter, v=1.0, D=1e-2):
    """(nc, nf, eta, xf0, workspace bytes) of a 1-D set-up (no GPU needed):
    coarse nodes x_k = k h_c, fine nodes x_i = xf0 + i h_f."""
    prm = Hyb1DParams(float(h_c), float(h_f), float(L_ov), int(max_iter), float(v), float(D))
    nc, nf, eta = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    xf0, ws = ctypes.c_double(), ctypes.c_size_t()
    rc = load().hyb1d_query(ctypes.addressof(prm), ctypes.addressof(nc), ctypes.addressof(nf), ctypes.addressof(eta),
                            ctypes.addressof(xf0), ctypes.addressof(ws))
    if rc != HYB_OK:
        raise HybError(rc, "hyb1d_query rejected the set-up")
    return nc.value, nf.value, eta.value, xf0.value, ws.value


class Hybrid1D:
    """The 1-D hybrid of Sec. 7.1 on the GPU (one workgroup per handle).
    ``initial(x)`` gives the initial concentration at host coordinates x
    (used on both grids)."""

    def __init__(self, h_c, h_f, L_ov, max_iter, initial, v=1.0, D=1e-2, device=None):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("Hybrid1D needs a GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.dev = torch.device(device or "cuda:0")
        self.nc, self.nf, self.eta, self.xf0, ws = hybrid1d_sizes(h_c, h_f, L_ov, max_iter, v, D)
        self.prm = Hyb1DParams(float(h_c), float(h_f), float(L_ov), int(max_iter), float(v), float(D))
        self.xc = np.arange(self.nc) * h_c
        self.xf = self.xf0 + np.arange(self.nf) * h_f
        self.dt_c = h_c ** 2 / (2.0 * D)
        d0 = np.ascontiguousarray(initial(self.xc), np.float64)
        u0 = np.ascontiguousarray(initial(self.xf), np.float64)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.dev)
        self.stream = torch.cuda.current_stream(self.dev)
        h = ctypes.c_void_p()
        rc = lib.hyb1d_create(ctypes.addressof(self.prm), _ptr(d0), _ptr(u0), self.ws.data_ptr(),
                              self.stream.cuda_stream, ctypes.addressof(h))
        if rc != HYB_OK:
            raise HybError(rc, "hyb1d_create failed (see stderr)")
        self.h = h
        _track(self)
        self.t = 0.0

    def run(self, n_steps):
        rc = load().hyb1d_run(self.h, int(n_steps))
        if rc != HYB_OK:
            raise HybError(rc, "hyb1d_run failed")
        self.t += n_steps * self.dt_c

    def state(self):
        """(coarse nodal values [nc], fine concentration [nf]) on the host."""
        d = np.empty(self.nc)
        u = np.empty(self.nf)
        rc = load().hyb1d_state(self.h, _ptr(d), _ptr(u))
        if rc != HYB_OK:
            raise HybError(rc, "hyb1d_state failed")
        return d, u

    def close(self):
        if getattr(self, "h", None):
            load().hyb1d_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has closed every live handle;
        # never call into the HIP runtime from a finaliser then (the check is
        # bound here: module globals such as sys may already be None)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
