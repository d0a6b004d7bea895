"""ctypes binding of ``librklpoisson.so`` (argument marshalling only).

Every numerical step runs in the library's HIP kernels; this module only turns
torch CUDA tensors into device pointers, options into the ``rkl_opts`` struct,
and status codes into exceptions.  There is no CPU fallback: if the library is
missing or no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from dataclasses import dataclass, field

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# RKL_LIB names another build of the same library (e.g. one compiled with
# different flags); the default is the in-tree build
LIB_PATH = os.environ.get("RKL_LIB") or os.path.join(_PKG, "librklpoisson.so")

RKL_OK, RKL_EINVAL, RKL_ENOMEM, RKL_ENOCONV, RKL_EDIVERGED, RKL_ENONFINITE, RKL_EHIP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "RKL_OK", -1: "RKL_EINVAL", -2: "RKL_ENOMEM", -3: "RKL_ENOCONV",
                -4: "RKL_EDIVERGED", -5: "RKL_ENONFINITE", -6: "RKL_EHIP"}
BC = {"dirichlet": 0, "periodic": 1}
PREC = {"fp64": 0, "mixed": 1}


class RKLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class c_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("bc", ctypes.c_int)]


class c_opts(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("tau_frac", ctypes.c_double), ("n_pre", ctypes.c_int),
                ("n_post", ctypes.c_int), ("min_coarse", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("prec", ctypes.c_int), ("four_pi_G", ctypes.c_double),
                ("coarse_tol", ctypes.c_double), ("coarse_max_steps", ctypes.c_int), ("smoother", ctypes.c_int),
                ("fuse", ctypes.c_int), ("zero_start", ctypes.c_int)]


class c_relax(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("s", ctypes.c_int), ("tau_frac", ctypes.c_double),
                ("omega", ctypes.c_double), ("tol_max", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("check_every", ctypes.c_int)]


class c_stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("levels", ctypes.c_int), ("res0", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("history_cap", ctypes.c_int), ("history_len", ctypes.c_int), ("status", ctypes.c_int)]


class c_tune(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc", ctypes.c_int),
                ("prec", ctypes.c_int), ("s", ctypes.c_int), ("variant", ctypes.c_int), ("target", ctypes.c_int),
                ("us", ctypes.c_double)]


EXPORTS = ("rkl_default_opts", "rkl_poisson_solve", "mg_vcycle", "rkl_smooth", "rkl_residual",
           "rkl_restrict", "rkl_prolong_add", "rkl_coarse_solve", "rkl_poisson_solve_batched",
           "rkl_tau_step_launches", "rkl_tune_set", "rkl_tune_clear", "rkl_tune_get", "rkl_autotune",
           "rkl_tune_set_s", "rkl_level_shapes", "rkl_variant_name", "rkl_gsrb_smooth", "rkl_default_relax_opts",
           "rkl_relax_solve", "rkl_gradient", "rkl_last_error", "rkl_release_all", "rkl_smooth_f32",
           "mg_vcycle_f32", "rkl_residual_f32", "rkl_restrict_f32", "rkl_prolong_add_f32", "rkl_coarse_solve_f32",
           "rkl_s_opt", "rkl_residual_noalloc")
SMOOTHERS = {"rkl": 0, "gsrb": 1}
RELAX = {"rkl": 0, "gsrb": 1, "sor": 2}
VARIANTS = {0: "heuristic", 1: "ring64x8", 2: "ring64x4", 3: "zq64x32", 4: "zq64x16", 5: "strip8x4",
            6: "strip8x1", 7: "strip4x4", 8: "strip2d8", 9: "strip2d4", 10: "strip5x1", 11: "stripyx8x4",
            12: "stripyx4x8", 13: "stripyx8x8", 14: "stripyx2x8", 15: "stripyx2x16"}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the shared library (no GPU needed) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2306_05332_amd.build` "
                          "(hipcc for gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    pg, po, ps = ctypes.POINTER(c_grid), ctypes.POINTER(c_opts), ctypes.POINTER(c_stats)
    lib.rkl_default_opts.argtypes = [po]
    lib.rkl_default_opts.restype = None
    lib.rkl_poisson_solve.argtypes = [pg, po, P, P, P, ps, P]
    lib.mg_vcycle.argtypes = [pg, po, P, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.rkl_smooth.argtypes = [pg, ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P, P, P]
    lib.rkl_residual.argtypes = [pg, P, P, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.rkl_restrict.argtypes = [pg, P, P, P]
    lib.rkl_prolong_add.argtypes = [pg, P, P, P]
    lib.rkl_coarse_solve.argtypes = [pg, po, P, P, ctypes.POINTER(ctypes.c_int), P]
    lib.rkl_poisson_solve_batched.argtypes = [pg, ctypes.c_int, po, ctypes.POINTER(P), ctypes.POINTER(P),
                                              ps, P]
    # float32 twins of the level building blocks (no face-data argument)
    lib.rkl_smooth_f32.argtypes = [pg, ctypes.c_int, ctypes.c_double, ctypes.c_int, P, P, P]
    lib.mg_vcycle_f32.argtypes = [pg, po, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.rkl_residual_f32.argtypes = [pg, P, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.rkl_restrict_f32.argtypes = [pg, P, P, P]
    lib.rkl_prolong_add_f32.argtypes = [pg, P, P, P]
    lib.rkl_coarse_solve_f32.argtypes = [pg, po, P, P, ctypes.POINTER(ctypes.c_int), P]
    for name in ("rkl_poisson_solve", "mg_vcycle", "rkl_smooth", "rkl_residual", "rkl_restrict",
                 "rkl_prolong_add", "rkl_coarse_solve", "rkl_poisson_solve_batched", "rkl_smooth_f32",
                 "mg_vcycle_f32", "rkl_residual_f32", "rkl_restrict_f32", "rkl_prolong_add_f32",
                 "rkl_coarse_solve_f32"):
        getattr(lib, name).restype = ctypes.c_int
    lib.rkl_tau_step_launches.argtypes = [pg, ctypes.c_int, ctypes.c_int]
    lib.rkl_tau_step_launches.restype = ctypes.c_int
    pt = ctypes.POINTER(c_tune)
    lib.rkl_tune_set.argtypes = [pt, ctypes.c_int]
    lib.rkl_tune_clear.argtypes = []
    lib.rkl_tune_get.argtypes = [pg, ctypes.c_int, ctypes.c_int, pt]
    lib.rkl_autotune.argtypes = [pg, ctypes.c_int, ctypes.c_int, ctypes.c_int, pt, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int), P]
    lib.rkl_tune_set_s.argtypes = [pg, ctypes.c_int, ctypes.c_int]
    lib.rkl_level_shapes.argtypes = [pg, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    for name in ("rkl_tune_set", "rkl_tune_clear", "rkl_tune_get", "rkl_autotune", "rkl_tune_set_s",
                 "rkl_level_shapes"):
        getattr(lib, name).restype = ctypes.c_int
    lib.rkl_variant_name.argtypes = [ctypes.c_int]
    lib.rkl_variant_name.restype = ctypes.c_char_p
    lib.rkl_gsrb_smooth.argtypes = [pg, ctypes.c_double, ctypes.c_int, P, P, P, P]
    lib.rkl_gsrb_smooth.restype = ctypes.c_int
    lib.rkl_default_relax_opts.argtypes = [ctypes.POINTER(c_relax)]
    lib.rkl_default_relax_opts.restype = None
    lib.rkl_relax_solve.argtypes = [pg, ctypes.POINTER(c_relax), P, P, P, ps, P]
    lib.rkl_relax_solve.restype = ctypes.c_int
    lib.rkl_residual_noalloc.argtypes = [pg, P, P, P, P, P, P]
    lib.rkl_residual_noalloc.restype = ctypes.c_int
    lib.rkl_s_opt.argtypes = [pg, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.rkl_s_opt.restype = ctypes.c_int
    lib.rkl_gradient.argtypes = [pg, P, P, P, P, P, P]
    lib.rkl_gradient.restype = ctypes.c_int
    lib.rkl_last_error.argtypes = []
    lib.rkl_last_error.restype = ctypes.c_char_p
    lib.rkl_release_all.argtypes = []
    lib.rkl_release_all.restype = None
    _lib = lib
    install_default_tuning()
    return lib


def install_default_tuning():
    """Install the stored tile table (``RKL_TUNING``: a path, or ``none``)."""
    path = os.environ.get("RKL_TUNING", "")
    if path.lower() == "none":
        return 0
    from . import autotune
    path = path or autotune.DEFAULT_TABLE
    return autotune.load(path) if os.path.exists(path) else 0


def _check(status):
    if status != RKL_OK:
        raise RKLError(status, _lib.rkl_last_error().decode())


@dataclass
class Options:
    """Mirror of ``rkl_opts`` with the library defaults."""

    s: int = 2
    tau_frac: float = 0.9
    n_pre: int = 2
    n_post: int = 1
    min_coarse: int = 4
    tol: float = 1e-10
    max_cycles: int = 100
    prec: str = "fp64"
    four_pi_G: float = 4.0 * math.pi
    coarse_tol: float = 0.0
    coarse_max_steps: int = 200
    smoother: str = "rkl"
    # transfer fusion where the strip kernel supports it: True / 3 both, 1 the
    # prolongation (into the first post-smoothing tau-step), 2 the restriction
    # (into the last pre-smoothing tau-step), False / 0 neither
    fuse: int = 3
    # rkl_poisson_solve starts from phi = 0 without reading phi (solve() sets
    # it when no phi0 is given)
    zero_start: bool = False

    def c(self):
        return c_opts(self.s, self.tau_frac, self.n_pre, self.n_post, self.min_coarse, self.tol,
                      self.max_cycles, PREC[self.prec], self.four_pi_G, self.coarse_tol,
                      self.coarse_max_steps, SMOOTHERS[self.smoother],
                      3 if self.fuse is True else int(self.fuse), int(self.zero_start))


@dataclass
class Stats:
    cycles: int = 0
    levels: int = 0
    res0: float = 0.0
    rel_res: float = 0.0
    history: list = field(default_factory=list)
    status: int = 0


def _grid(shape, h, bc):
    """rkl_grid of a (nz, ny, nx) or two-dimensional (ny, nx) array.  A 2-D
    problem is the single layer nz = 1 with hz = inf (no z coupling); h may
    then be (hx, hy) or one number."""
    flat = len(shape) == 2
    if flat:
        shape = (1,) + tuple(shape)
    nz, ny, nx = shape
    if isinstance(h, (int, float)):
        h = (float(h), float(h), math.inf if flat else float(h))
    elif len(h) == 2:
        h = (h[0], h[1], math.inf)
    return c_grid(nx, ny, nz, float(h[0]), float(h[1]), float(h[2]), BC[bc])


def _flat_shape(t):
    """A fine array of one z plane is two-dimensional for the transfer operators."""
    return t.dim() == 2 or t.shape[0] == 1


def _dev(t, name, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _current_stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def pack_faces(faces, device=None):
    """Six face arrays (x-, x+, y-, y+, z-, z+) -> one flat float64 CUDA tensor.
    Four arrays (x-, x+ of ny values; y-, y+ of nx values) describe a 2-D grid:
    its two z faces carry no weight and are packed as zeros."""
    parts = [torch.as_tensor(f, dtype=torch.float64).reshape(-1) for f in faces]
    if len(parts) == 4:
        nxy = parts[0].numel() * parts[2].numel()
        parts += [torch.zeros(nxy, dtype=torch.float64), torch.zeros(nxy, dtype=torch.float64)]
    out = torch.cat(parts)
    return out.to(device or "cuda").contiguous()


def _check_faces(faces, shape, bc):
    if faces is None:
        return
    if bc != "dirichlet":
        raise ValueError("faces are only valid for Dirichlet grids")
    nz, ny, nx = (1,) + tuple(shape) if len(shape) == 2 else shape
    want = 2 * (ny * nz + nx * nz + nx * ny)
    if faces.numel() != want:
        raise ValueError(f"packed faces must hold {want} values for shape {tuple(shape)}, got {faces.numel()}")


def solve(rho, h, bc="periodic", faces=None, phi0=None, opts: Options | None = None,
          history_cap=256, raise_on_error=True):
    """phi solving nabla^2 phi = four_pi_G rho (rkl_poisson_solve).  rho: (nz, ny, nx)
    float64 CUDA tensor.  Returns (phi, Stats)."""
    lib = load_library()
    opts = opts or Options()
    if phi0 is None:
        # a cold start: the library does not read phi's contents.  phi is
        # still zero-filled here (one fill kernel, mostly hidden behind the
        # call's host work): with uninitialised outputs a later standalone
        # tau-step sweep in the same process ran 8-12 % slower (measured, not
        # explained)
        phi = torch.zeros_like(rho)
        opts = dataclasses.replace(opts, zero_start=True)
    else:
        phi = phi0.clone()
    _check_faces(faces, rho.shape, bc)
    g = _grid(rho.shape, h, bc)
    hist = (ctypes.c_double * max(1, history_cap))()
    st = c_stats(0, 0, 0.0, 0.0, hist, history_cap, 0, 0)
    co = opts.c()
    status = lib.rkl_poisson_solve(ctypes.byref(g), ctypes.byref(co), _dev(rho, "rho"), _dev(faces, "faces"),
                                   _dev(phi, "phi"), ctypes.byref(st), _stream(rho))
    stats = Stats(st.cycles, st.levels, st.res0, st.rel_res, list(hist[:st.history_len]), status)
    if raise_on_error and status != RKL_OK:
        _check(status)
    return phi, stats


def _is_f32(t):
    """float32 arrays take the float32 entry points (the mixed path's kernels,
    error-equation ghosts, no face data)."""
    return isinstance(t, torch.Tensor) and t.dtype == torch.float32


def _no_faces_f32(faces):
    if faces is not None:
        raise ValueError("the float32 entry points take no face data (homogeneous or periodic ghosts)")


def vcycle(f, phi, h, bc="periodic", faces=None, opts: Options | None = None, want_residual=False):
    """One V-cycle on M phi = f in place (mg_vcycle; float32 arrays: mg_vcycle_f32);
    returns the relative residual or None."""
    lib = load_library()
    opts = opts or Options()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    co = opts.c()
    rel = ctypes.c_double(0.0)
    relp = ctypes.byref(rel) if want_residual else None
    if _is_f32(f):
        _no_faces_f32(faces)
        _check(lib.mg_vcycle_f32(ctypes.byref(g), ctypes.byref(co), _dev(f, "f", torch.float32),
                                 _dev(phi, "phi", torch.float32), relp, _stream(f)))
    else:
        _check(lib.mg_vcycle(ctypes.byref(g), ctypes.byref(co), _dev(f, "f"), _dev(faces, "faces"),
                             _dev(phi, "phi"), relp, _stream(f)))
    return rel.value if want_residual else None


def smooth(f, phi, h, bc="periodic", s=2, tau_frac=0.9, n_steps=1, faces=None):
    """n_steps RKL tau-steps on M phi = f in place (rkl_smooth; float32 arrays: rkl_smooth_f32)."""
    lib = load_library()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    if _is_f32(f):
        _no_faces_f32(faces)
        _check(lib.rkl_smooth_f32(ctypes.byref(g), int(s), float(tau_frac), int(n_steps),
                                  _dev(f, "f", torch.float32), _dev(phi, "phi", torch.float32), _stream(f)))
        return phi
    _check(lib.rkl_smooth(ctypes.byref(g), int(s), float(tau_frac), int(n_steps), _dev(f, "f"),
                          _dev(faces, "faces"), _dev(phi, "phi"), _stream(f)))
    return phi


def residual(f, phi, h, bc="periodic", faces=None):
    """(f - M phi, ||f - M phi||_2) (rkl_residual; float32 arrays: rkl_residual_f32)."""
    lib = load_library()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    r = torch.empty_like(f)
    nrm = ctypes.c_double(0.0)
    if _is_f32(f):
        _no_faces_f32(faces)
        _check(lib.rkl_residual_f32(ctypes.byref(g), _dev(f, "f", torch.float32), _dev(phi, "phi", torch.float32),
                                    _dev(r, "r", torch.float32), ctypes.byref(nrm), _stream(f)))
        return r, nrm.value
    _check(lib.rkl_residual(ctypes.byref(g), _dev(f, "f"), _dev(faces, "faces"), _dev(phi, "phi"),
                            _dev(r, "r"), ctypes.byref(nrm), _stream(f)))
    return r, nrm.value


def residual_noalloc(f, phi, h, bc="periodic", faces=None):
    """(f - M phi, ||f - M phi||_2 as a one-element device tensor) through
    rkl_residual_noalloc: no device allocation in the library and no
    synchronisation (the outputs are allocated here, by the caller's side)."""
    lib = load_library()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    r = torch.empty_like(f)
    nrm = torch.empty(1, dtype=torch.float64, device=f.device)
    _check(lib.rkl_residual_noalloc(ctypes.byref(g), _dev(f, "f"), _dev(faces, "faces"), _dev(phi, "phi"),
                                    _dev(r, "r"), _dev(nrm, "norm"), _stream(f)))
    return r, nrm


def restrict(fine):
    """coarse = R(fine): 8-point average, or the 4-point one of a 2-D (ny, nx)
    or (1, ny, nx) array (rkl_restrict; float32 arrays: rkl_restrict_f32)."""
    lib = load_library()
    flat = _flat_shape(fine)
    ny, nx = fine.shape[-2:]
    cshape = (ny // 2, nx // 2) if fine.dim() == 2 else (1 if flat else fine.shape[0] // 2, ny // 2, nx // 2)
    coarse = torch.empty(cshape, dtype=fine.dtype, device=fine.device)
    g = _grid(fine.shape, (1.0, 1.0) if flat else 1.0, "periodic")
    fn, dt = (lib.rkl_restrict_f32, torch.float32) if _is_f32(fine) else (lib.rkl_restrict, torch.float64)
    _check(fn(ctypes.byref(g), _dev(fine, "fine", dt), _dev(coarse, "coarse", dt), _stream(fine)))
    return coarse


def prolong_add(coarse, fine, bc="periodic"):
    """fine += P(coarse): trilinear, or bilinear for a 2-D fine array
    (rkl_prolong_add; float32 arrays: rkl_prolong_add_f32)."""
    lib = load_library()
    g = _grid(fine.shape, (1.0, 1.0) if _flat_shape(fine) else 1.0, bc)
    fn, dt = (lib.rkl_prolong_add_f32, torch.float32) if _is_f32(fine) else (lib.rkl_prolong_add, torch.float64)
    _check(fn(ctypes.byref(g), _dev(coarse, "coarse", dt), _dev(fine, "fine", dt), _stream(fine)))
    return fine


def coarse_solve(b, h, bc="periodic", opts: Options | None = None):
    """Accelerated RKL solve of M u = b with homogeneous/periodic ghosts
    (rkl_coarse_solve; float32 arrays: rkl_coarse_solve_f32)."""
    lib = load_library()
    opts = opts or Options()
    g = _grid(b.shape, h, bc)
    u = torch.empty_like(b)
    steps = ctypes.c_int(0)
    co = opts.c()
    fn, dt = (lib.rkl_coarse_solve_f32, torch.float32) if _is_f32(b) else (lib.rkl_coarse_solve, torch.float64)
    _check(fn(ctypes.byref(g), ctypes.byref(co), _dev(b, "b", dt), _dev(u, "u", dt), ctypes.byref(steps),
              _stream(b)))
    return u, steps.value


def solve_batched(rhos, hs, bcs, opts: Options | None = None, history_cap=64, raise_on_error=True):
    """Batched solve of independent problems (rkl_poisson_solve_batched).
    rhos: list of float64 CUDA tensors (sizes may differ), hs: spacing per
    member, bcs: one boundary type or one per member.  Returns (phis, stats
    list); each Stats carries its member's own status."""
    lib = load_library()
    opts = opts or Options()
    n = len(rhos)
    if isinstance(bcs, str):
        bcs = [bcs] * n
    if len(hs) != n or len(bcs) != n:
        raise ValueError("rhos, hs and bcs must have the same length")
    if n == 0:
        return [], []
    grids = (c_grid * n)(*[_grid(r.shape, h, b) for r, h, b in zip(rhos, hs, bcs)])
    phis = [torch.zeros_like(r) for r in rhos]
    rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
    pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in phis])
    for r in rhos:
        _dev(r, "rho")
    hists = [(ctypes.c_double * history_cap)() for _ in range(n)]
    sts = (c_stats * n)(*[c_stats(0, 0, 0.0, 0.0, hh, history_cap, 0, 0) for hh in hists])
    co = opts.c()
    status = lib.rkl_poisson_solve_batched(grids, n, ctypes.byref(co), rp, pp, sts, _stream(rhos[0]))
    if status in (RKL_EINVAL, RKL_ENOMEM, RKL_EHIP) or (raise_on_error and status != RKL_OK):
        _check(status)
    stats = [Stats(s.cycles, s.levels, s.res0, s.rel_res, list(hh[:s.history_len]), s.status)
             for s, hh in zip(sts, hists)]
    return phis, stats


def gsrb_smooth(f, phi, h, bc="periodic", omega=1.0, n_iter=1, faces=None):
    """n_iter red-black Gauss-Seidel (omega = 1) or SOR passes on M phi = f in place (rkl_gsrb_smooth)."""
    lib = load_library()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    _check(lib.rkl_gsrb_smooth(ctypes.byref(g), float(omega), int(n_iter), _dev(f, "f"), _dev(faces, "faces"),
                               _dev(phi, "phi"), _stream(f)))
    return phi


def relax_solve(f, h, bc="dirichlet", method="rkl", faces=None, phi0=None, s=0, tau_frac=0.9, omega=0.0,
                tol_max=1e-10, max_iters=100000, check_every=1, history_cap=4096, raise_on_error=True):
    """Single-level relaxation to max|M phi - f| <= tol_max (rkl_relax_solve, App. B).
    method: "rkl" (s = 0: accelerated schedule; s = -1: the App. A.3 fixed count, see s_opt),
    "gsrb" or "sor" (omega = 0: App. B optimum).
    Returns (phi, Stats) with Stats.cycles = iterations, Stats.rel_res = final max residual."""
    lib = load_library()
    _check_faces(faces, f.shape, bc)
    g = _grid(f.shape, h, bc)
    phi = torch.zeros_like(f) if phi0 is None else phi0.clone()
    ro = c_relax(RELAX[method], int(s), float(tau_frac), float(omega), float(tol_max), int(max_iters),
                 int(check_every))
    hist = (ctypes.c_double * max(1, history_cap))()
    st = c_stats(0, 0, 0.0, 0.0, hist, history_cap, 0, 0)
    status = lib.rkl_relax_solve(ctypes.byref(g), ctypes.byref(ro), _dev(f, "f"), _dev(faces, "faces"),
                                 _dev(phi, "phi"), ctypes.byref(st), _stream(f))
    stats = Stats(st.cycles, st.levels, st.res0, st.rel_res, list(hist[:st.history_len]), status)
    if status in (RKL_EINVAL, RKL_ENOMEM, RKL_EHIP) or (raise_on_error and status != RKL_OK):
        _check(status)
    return phi, stats


def s_opt(shape, h, bc="dirichlet", tau_frac=0.9, kmax=6, digits=2.0):
    """Best fixed RKL stage count of App. A.3 for single-level relaxation on a
    grid of shape (nz, ny, nx) or (ny, nx) (rkl_s_opt; host arithmetic, no
    GPU).  Returns (s_opt, m_eff)."""
    lib = load_library()
    m = ctypes.c_double(0.0)
    r = lib.rkl_s_opt(ctypes.byref(_grid(shape, h, bc)), float(tau_frac), int(kmax), float(digits),
                      ctypes.byref(m))
    if r < 0:
        _check(r)
    return r, m.value


def gradient(phi, h, bc="periodic", faces=None):
    """(g_x, g_y, g_z) = -grad(phi) by 4th-order differences (rkl_gradient)."""
    lib = load_library()
    _check_faces(faces, phi.shape, bc)
    g = _grid(phi.shape, h, bc)
    gx, gy, gz = (torch.empty_like(phi) for _ in range(3))
    _check(lib.rkl_gradient(ctypes.byref(g), _dev(phi, "phi"), _dev(faces, "faces"), _dev(gx, "gx"), _dev(gy, "gy"),
                            _dev(gz, "gz"), _stream(phi)))
    return gx, gy, gz


def tau_step_launches(shape, s, bc="periodic", prec="fp64", h=1.0):
    """Kernel launches per finest-level tau-step (1 = fused single pass).  A
    (ny, nx) shape, or h = (hx, hy) / hz = inf, is a two-dimensional level."""
    lib = load_library()
    g = _grid(shape, h, bc)
    r = lib.rkl_tau_step_launches(ctypes.byref(g), int(s), PREC[prec])
    if r < 0:
        _check(r)
    return r


def kernel_info(shape, s, bc="periodic", prec="fp64", h=1.0):
    """Algorithmic HBM bytes of the finest-level sweep kernel, per launch.

    Fused tau-step: u and b read once, Y_s written once: 3 words per cell.
    Per-stage kernels: stage 1 moves 3 words per cell (Y_0, b in; Y_1 out),
    stages j >= 2 move 4 (Y_{j-1}, Y_{j-2}, b in; Y_j out); the per-launch
    figure is their mean over the s launches of one tau-step.
    """
    cells = math.prod(shape)
    word = 8 if prec == "fp64" else 4
    launches = tau_step_launches(shape, s, bc, prec, h)
    tname = "double" if prec == "fp64" else "float"
    if launches == 1:
        words = 3.0
        v = tune_get(shape, s, bc, prec, h)
        name = {"zq64x32": f"k_tau_zq<{tname}, {s}, 64, 32>", "zq64x16": f"k_tau_zq<{tname}, {s}, 64, 16>",
                "ring64x4": f"k_fused_tau<{tname}, {s}, 64, 4>", "strip8x4": f"k_tau_strip<{tname}, {s}, 8, 4>",
                "strip8x1": f"k_tau_strip<{tname}, {s}, 8, 1>", "strip4x4": f"k_tau_strip<{tname}, {s}, 4, 4>",
                "strip2d8": f"k_tau_strip<{tname}, {s}, 8, 1>", "strip2d4": f"k_tau_strip<{tname}, {s}, 4, 1>",
                "strip5x1": f"k_tau_strip<{tname}, {s}, 5, 1>",
                "stripyx8x4": f"k_tau_strip_yx<{tname}, {s}, 8, 4>",
                "stripyx4x8": f"k_tau_strip_yx<{tname}, {s}, 4, 8>",
                "stripyx8x8": f"k_tau_strip_yx<{tname}, {s}, 8, 8>",
                "stripyx2x8": f"k_tau_strip_yx<{tname}, {s}, 2, 8>",
                "stripyx2x16": f"k_tau_strip_yx<{tname}, {s}, 2, 16>",
                }.get(v["variant"], f"k_fused_tau<{tname}, {s}, 64, 8>")
    else:
        words = (3.0 + 4.0 * (s - 1)) / s
        name = f"k_stage<{tname}>"
    return {"kernel": name, "launches_per_tau": launches, "bytes_per_launch": words * word * cells,
            "words_per_cell_launch": words}


# ---------------------------------------------------------------- tuning
BC_NAMES = {v: k for k, v in BC.items()}
PREC_NAMES = {v: k for k, v in PREC.items()}


def _entry_dict(e):
    return {"nx": e.nx, "ny": e.ny, "nz": e.nz, "bc": BC_NAMES[e.bc], "prec": PREC_NAMES[e.prec], "s": e.s,
            "variant": VARIANTS.get(e.variant, str(e.variant)), "target": e.target, "us": e.us}


def _entry_c(d):
    inv = {v: k for k, v in VARIANTS.items()}
    var = d["variant"]
    var = inv[var] if isinstance(var, str) else int(var)
    return c_tune(int(d["nx"]), int(d["ny"]), int(d["nz"]), BC[d["bc"]], PREC[d["prec"]], int(d["s"]), var,
                  int(d.get("target", 0)), float(d.get("us", 0.0)))


def tune_set(entries):
    """Install tile choices (dicts as returned by autotune_level / tune_get)."""
    lib = load_library()
    arr = (c_tune * max(1, len(entries)))(*[_entry_c(d) for d in entries])
    _check(lib.rkl_tune_set(arr, len(entries)))


def tune_clear():
    _check(load_library().rkl_tune_clear())


def tune_get(shape, s, bc="periodic", prec="fp64", h=1.0):
    """The tile choice in effect for a level of shape (nz, ny, nx) (or a 2-D
    (ny, nx) level; h = (hx, hy) marks a (1, ny, nx) shape as 2-D too)."""
    lib = load_library()
    out = c_tune()
    _check(lib.rkl_tune_get(ctypes.byref(_grid(shape, h, bc)), int(s), PREC[prec], ctypes.byref(out)))
    return _entry_dict(out)


def autotune_level(shape, s, bc="periodic", prec="fp64", reps=20, h=1.0):
    """Time every variant/target on one level (GPU); installs the fastest and
    returns all measurements, fastest first."""
    lib = load_library()
    cap = 4096
    res = (c_tune * cap)()
    n = ctypes.c_int(0)
    _check(lib.rkl_autotune(ctypes.byref(_grid(shape, h, bc)), int(s), PREC[prec], int(reps), res, cap,
                            ctypes.byref(n), _current_stream()))
    return [_entry_dict(res[q]) for q in range(min(n.value, cap))]


def tune_set_s(shape, s, bc="periodic", prec="fp64"):
    """Stage count used for this grid when Options.s == 0 (0 erases)."""
    lib = load_library()
    _check(lib.rkl_tune_set_s(ctypes.byref(_grid(shape, 1.0, bc)), PREC[prec], int(s)))


def level_shapes(shape, min_coarse=4, bc="periodic", h=1.0):
    """Multigrid level shapes (nz, ny, nx), finest first.  A (ny, nx) shape, or
    h = (hx, hy), describes a two-dimensional grid."""
    lib = load_library()
    buf = (ctypes.c_int * (3 * 64))()
    L = lib.rkl_level_shapes(ctypes.byref(_grid(shape, h, bc)), int(min_coarse), buf, 64)
    if L < 0:
        _check(L)
    return [(buf[3 * q + 2], buf[3 * q + 1], buf[3 * q]) for q in range(min(L, 64))]


def release_all():
    load_library().rkl_release_all()
