"""Thin ctypes binding of libbsex.so (the C ABI declared in include/bsex.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch CUDA tensors (float64, contiguous) on the
library's device; host arrays are numpy.  The library must be built
(``python -m paper_2607_20728_amd.build`` or ``__graft_entry__.build()``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsex.so")

ABI_VERSION = 4
OK, EINVAL, ENOMEM, EHIP, ENOCONV, EGAP, EABI, ESTATE = range(8)
K_D, K_1E, K_1D_BARE, K_1D_PDEP, K_ALL = 1, 2, 4, 8, 15
FP64, MIXED = 0, 1
TAU_AUTO, TAU_CACHE, TAU_REBUILD = 0, 1, 2

SYMBOLS = ("bse_abi_version", "bse_last_error", "bse_warm_up", "bse_basis_size", "bse_basis_gvectors",
           "bse_init_system", "bse_get_info", "bse_get_orbitals", "bse_get_frame", "bse_apply",
           "bse_davidson", "bse_apply_coupling", "bse_full_bse", "bse_u_vector", "bse_zvector_solve", "bse_forces", "bse_forces_noalloc",
           "bse_ground_state_forces",
           "bse_set_precision", "bse_set_profiling", "bse_get_phase_times",
           "bse_mlp_create", "bse_mlp_n_params", "bse_mlp_set_params", "bse_mlp_get_params",
           "bse_mlp_set_norm", "bse_mlp_forward", "bse_mlp_train_step", "bse_mlp_free",
           "bse_set_learned", "bse_learned_features", "bse_set_graphs", "bse_batch_run",
           "bse_tune_cache_clear", "bse_free", "bse_memory_cache")
LEARN_NFEAT, LEARN_NOUT = 8, 2


class BseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bsex error {code}: {msg}")
        self.code = code


class SystemDesc(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("cell", C.c_double * 3), ("grid", C.c_int32 * 3),
                ("ecut", C.c_double), ("n_sites", C.c_int32),
                ("site_xyz", C.POINTER(C.c_double)), ("site_depth", C.POINTER(C.c_double)),
                ("site_width", C.POINTER(C.c_double)), ("n_val", C.c_int32),
                ("n_pdep", C.c_int32), ("pdep", C.POINTER(C.c_double)),
                ("lambda_", C.POINTER(C.c_double)), ("scissor", C.c_double),
                ("spin_factor", C.c_double), ("precision", C.c_int32),
                ("tau_policy", C.c_int32), ("tau_budget_bytes", C.c_int64),
                ("gap_min", C.c_double), ("kernel_mask", C.c_int32), ("n_orb", C.c_int32),
                ("orbitals", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
                ("n_extra", C.c_int32), ("gs_tol", C.c_double), ("stream", C.c_void_p),
                ("ks_model", C.c_int32), ("rho_floor", C.c_double), ("scf_tol", C.c_double),
                ("alpha_exx", C.c_double), ("localize", C.c_int32),
                ("prune_threshold", C.c_double), ("loc_rotation", C.POINTER(C.c_double)),
                ("loc_max_sweeps", C.c_int32), ("loc_tol", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_pw", C.c_int32), ("n_val", C.c_int32), ("n_pdep", C.c_int32),
                ("n_orb", C.c_int32), ("grid", C.c_int32 * 3), ("tau_policy", C.c_int32),
                ("tau_blocks", C.c_int64), ("tau_blocks_cached", C.c_int64),
                ("tau_bytes", C.c_int64), ("gs_resid", C.c_double), ("ks_gap", C.c_double),
                ("precision", C.c_int32), ("active_precision", C.c_int32),
                ("tau_bytes_f32", C.c_int64), ("gs_sweeps", C.c_int32),
                ("t_ground_state_ms", C.c_double), ("t_tau_ms", C.c_double),
                ("t_tau_alloc_ms", C.c_double), ("t_init_ms", C.c_double),
                ("scf_iters", C.c_int32), ("scf_resid", C.c_double),
                ("tau_blocks_all", C.c_int64), ("loc_spread", C.c_double),
                ("loc_sweeps", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("precision", C.c_int32), ("n_streams", C.c_int32),
                ("mem_budget", C.c_int64), ("autotune", C.c_int32), ("use_graph", C.c_int32)]


class BatchResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("omega", C.c_double),
                ("dwdR_host", C.POINTER(C.c_double)), ("davidson_iters", C.c_int32),
                ("z_iters", C.c_int32), ("t_init_ms", C.c_double), ("t_davidson_ms", C.c_double),
                ("t_z_ms", C.c_double), ("t_force_ms", C.c_double), ("variant", C.c_int32),
                ("stream_slot", C.c_int32), ("message", C.c_char * 160)]


class SolverOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("block", C.c_int32),
                ("max_subspace", C.c_int32), ("x0_dev", C.c_void_p), ("n_x0", C.c_int32),
                ("z0_dev", C.c_void_p), ("use_learned", C.c_int32),
                ("precond_shift_host", C.POINTER(C.c_double)),
                ("band_iters_host", C.POINTER(C.c_int32)), ("two_level", C.c_int32)]


class SolverStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("applies", C.c_int32), ("resid", C.c_double * 16),
                ("t_ms", C.c_double), ("applies_fp64", C.c_int32), ("learned", C.c_int32),
                ("fallback", C.c_int32), ("t_u_ms", C.c_double)]


class PhaseTimes(C.Structure):
    _fields_ = [("n_phase", C.c_int32), ("name", C.c_char_p * 16), ("ms", C.c_double * 16),
                ("count", C.c_int64 * 16)]


_lib = None


def lib():
    """Load libbsex.so once; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2607_20728_amd.build`")
    L = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    L.bse_abi_version.restype = C.c_int32
    L.bse_last_error.restype = C.c_char_p
    L.bse_basis_size.argtypes = [dp, C.POINTER(C.c_int32), C.c_double, C.POINTER(C.c_int32)]
    L.bse_basis_gvectors.argtypes = [dp, C.POINTER(C.c_int32), C.c_double,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int8)]
    L.bse_init_system.argtypes = [C.POINTER(SystemDesc), C.POINTER(C.c_void_p)]
    L.bse_get_info.argtypes = [C.c_void_p, C.POINTER(Info)]
    L.bse_get_orbitals.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, dp]
    L.bse_get_frame.argtypes = [C.c_void_p, dp, dp]
    L.bse_apply.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    L.bse_davidson.argtypes = [C.c_void_p, C.c_int32, C.POINTER(SolverOpts), dp, C.c_void_p,
                               C.POINTER(SolverStats)]
    L.bse_u_vector.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.bse_apply_coupling.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    L.bse_full_bse.argtypes = [C.c_void_p, C.c_int32, C.POINTER(SolverOpts), dp, C.c_void_p,
                               C.c_void_p, C.POINTER(SolverStats)]
    L.bse_zvector_solve.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(SolverOpts), C.c_void_p,
                                    C.POINTER(SolverStats)]
    L.bse_forces.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, dp]
    L.bse_forces_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.bse_ground_state_forces.argtypes = [C.c_void_p, dp]
    L.bse_set_precision.argtypes = [C.c_void_p, C.c_int32]
    L.bse_memory_cache.argtypes = [C.c_int32]
    fp = C.POINTER(C.c_float)
    L.bse_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_uint64, C.c_void_p,
                                 C.POINTER(C.c_void_p)]
    L.bse_mlp_n_params.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
    L.bse_mlp_set_params.argtypes = [C.c_void_p, fp]
    L.bse_mlp_get_params.argtypes = [C.c_void_p, fp]
    L.bse_mlp_set_norm.argtypes = [C.c_void_p, fp, fp, fp, fp]
    L.bse_mlp_forward.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    L.bse_mlp_train_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_float, fp, C.c_void_p]
    L.bse_mlp_free.argtypes = [C.c_void_p]
    L.bse_set_learned.argtypes = [C.c_void_p, C.c_void_p]
    L.bse_set_graphs.argtypes = [C.c_void_p, C.c_int32]
    L.bse_batch_run.argtypes = [C.POINTER(SystemDesc), C.c_int32, C.POINTER(BatchOpts),
                                C.POINTER(BatchResult)]
    L.bse_learned_features.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, fp, dp]
    L.bse_set_profiling.argtypes = [C.c_void_p, C.c_int32]
    L.bse_get_phase_times.argtypes = [C.c_void_p, C.POINTER(PhaseTimes), C.c_int32]
    L.bse_free.argtypes = [C.c_void_p]
    if L.bse_abi_version() != ABI_VERSION:
        raise RuntimeError("libbsex ABI version mismatch")
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        raise BseError(rc, lib().bse_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
def basis_size(cell, grid, ecut):
    c = _f64(cell)
    g = np.ascontiguousarray(grid, dtype=np.int32)
    n = C.c_int32()
    _check(lib().bse_basis_size(_dptr(c), g.ctypes.data_as(C.POINTER(C.c_int32)), float(ecut),
                                C.byref(n)))
    return n.value


def basis_gvectors(cell, grid, ecut):
    n = basis_size(cell, grid, ecut)
    c = _f64(cell)
    g = np.ascontiguousarray(grid, dtype=np.int32)
    mill = np.zeros((n, 3), dtype=np.int32)
    kind = np.zeros(n, dtype=np.int8)
    _check(lib().bse_basis_gvectors(_dptr(c), g.ctypes.data_as(C.POINTER(C.c_int32)),
                                    float(ecut), mill.ctypes.data_as(C.POINTER(C.c_int32)),
                                    kind.ctypes.data_as(C.POINTER(C.c_int8))))
    return mill, kind


class Context:
    """Owns one bse_ctx; host inputs are kept alive for the init call only."""

    def __init__(self, handle):
        self.h = C.c_void_p(handle)

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.bse_free(h)
            self.h = C.c_void_p(None)


def init_system(cell, grid, ecut, site_xyz, site_depth, site_width, n_val, pdep, lam, *,
                scissor=0.0, spin_factor=2.0, tau_policy=TAU_AUTO, tau_budget_bytes=0,
                gap_min=0.0, kernel_mask=K_ALL, orbitals=None, eps=None, n_extra=8,
                gs_tol=1e-10, precision=FP64, stream=None, desc_only=False, ks_model=0,
                rho_floor=0.0, scf_tol=0.0, alpha_exx=0.0, localize=0, prune_threshold=0.0,
                loc_rotation=None, loc_max_sweeps=0, loc_tol=0.0):
    """bse_init_system.  orbitals [n_orb][n_pw] / eps [n_orb] (host) or None to
    let the library solve the ground state."""
    import torch
    xyz, dep, wid = _f64(site_xyz).reshape(-1, 3), _f64(site_depth), _f64(site_width)
    P, lm = _f64(pdep), _f64(lam)
    d = SystemDesc()
    d.abi_version = ABI_VERSION
    d.cell[:] = [float(x) for x in cell]
    d.grid[:] = [int(x) for x in grid]
    d.ecut = float(ecut)
    d.n_sites = len(dep)
    d.site_xyz, d.site_depth, d.site_width = _dptr(xyz), _dptr(dep), _dptr(wid)
    d.n_val = int(n_val)
    d.n_pdep = P.shape[1] if P.ndim == 2 else 0
    d.pdep, d.lambda_ = _dptr(P), _dptr(lm)
    d.scissor = float(scissor)
    d.spin_factor = float(spin_factor)
    d.precision = int(precision)
    d.tau_policy = int(tau_policy)
    d.tau_budget_bytes = int(tau_budget_bytes)
    d.gap_min = float(gap_min)
    d.kernel_mask = int(kernel_mask)
    keep = [xyz, dep, wid, P, lm]
    if orbitals is not None:
        O, E = _f64(orbitals), _f64(eps)
        keep += [O, E]
        d.n_orb = O.shape[0]
        d.orbitals, d.eps = _dptr(O), _dptr(E)
    d.n_extra = int(n_extra)
    d.gs_tol = float(gs_tol)
    d.ks_model = int(ks_model)
    d.rho_floor = float(rho_floor)
    d.scf_tol = float(scf_tol)
    d.alpha_exx = float(alpha_exx)
    d.localize = int(localize)
    d.prune_threshold = float(prune_threshold)
    if loc_rotation is not None:
        Ur = _f64(loc_rotation)
        keep.append(Ur)
        d.loc_rotation = _dptr(Ur)
    d.loc_max_sweeps = int(loc_max_sweeps)
    d.loc_tol = float(loc_tol)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    d.stream = C.c_void_p(stream)
    if desc_only:
        return d, keep
    h = C.c_void_p()
    _check(lib().bse_init_system(C.byref(d), C.byref(h)))
    ctx = Context(h.value)
    return ctx


def init_from_synth(sysd, **kw):
    """init_system from a ``synth.make_system`` dict."""
    return init_system(sysd["cell"], sysd["grid"], sysd["ecut"], sysd["site_xyz"],
                       sysd["site_depth"], sysd["site_width"], sysd["n_val"], sysd["pdep"],
                       sysd["lam"], **kw)


def batch_run(systems, *, tol=1e-6, precision=FP64, n_streams=4, mem_budget=0, autotune=True,
              use_graph=True, check=True):
    """bse_batch_run over synth.make_system dicts (library ground states).
    Returns a list of per-system dicts (omega, dwdR, iterations, times)."""
    n = len(systems)
    descs = (SystemDesc * n)()
    keep = []
    res = (BatchResult * n)()
    outs = []
    for i, sd in enumerate(systems):
        d, k = init_system(sd["cell"], sd["grid"], sd["ecut"], sd["site_xyz"], sd["site_depth"],
                           sd["site_width"], sd["n_val"], sd["pdep"], sd["lam"], n_extra=8,
                           desc_only=True, stream=0)
        descs[i] = d
        keep.append(k)
        f = np.zeros((max(len(sd["site_depth"]), 1), 3))
        outs.append(f)
        res[i].dwdR_host = _dptr(f)
    o = BatchOpts(float(tol), int(precision), int(n_streams), int(mem_budget),
                  1 if autotune else 0, 1 if use_graph else 0)
    rc = lib().bse_batch_run(descs, n, C.byref(o), res)
    if check:
        _check(rc)
    out = []
    for i in range(n):
        r = res[i]
        out.append(dict(status=r.status, omega=r.omega, dwdR=outs[i][:len(systems[i]["site_depth"])],
                        davidson_iters=r.davidson_iters, z_iters=r.z_iters,
                        t_init_ms=r.t_init_ms, t_davidson_ms=r.t_davidson_ms, t_z_ms=r.t_z_ms,
                        t_force_ms=r.t_force_ms, variant=r.variant, stream=r.stream_slot,
                        message=r.message.decode()))
    return out


def tune_cache_clear():
    _check(lib().bse_tune_cache_clear())


def get_info(ctx):
    i = Info()
    _check(lib().bse_get_info(ctx.h, C.byref(i)))
    return dict(n_pw=i.n_pw, n_val=i.n_val, n_pdep=i.n_pdep, n_orb=i.n_orb, grid=tuple(i.grid),
                tau_policy=i.tau_policy, tau_blocks=i.tau_blocks,
                tau_blocks_cached=i.tau_blocks_cached, tau_bytes=i.tau_bytes,
                gs_resid=i.gs_resid, ks_gap=i.ks_gap, precision=i.precision,
                active_precision=i.active_precision, tau_bytes_f32=i.tau_bytes_f32,
                gs_sweeps=i.gs_sweeps, t_ground_state_ms=i.t_ground_state_ms,
                t_tau_ms=i.t_tau_ms, t_tau_alloc_ms=i.t_tau_alloc_ms, t_init_ms=i.t_init_ms,
                scf_iters=i.scf_iters, scf_resid=i.scf_resid, tau_blocks_all=i.tau_blocks_all,
                loc_spread=i.loc_spread, loc_sweeps=i.loc_sweeps)


def get_frame(ctx):
    """bse_get_frame: (U [n_val][n_val], centres [n_val][3]) of a localised
    context."""
    n = get_info(ctx)["n_val"]
    U = np.zeros((n, n))
    cen = np.zeros((n, 3))
    _check(lib().bse_get_frame(ctx.h, _dptr(U), _dptr(cen)))
    return U, cen


def get_orbitals(ctx, n=None):
    import torch
    info = get_info(ctx)
    n = info["n_val"] if n is None else n
    out = torch.empty((n, info["n_pw"]), dtype=torch.float64, device="cuda")
    e = np.zeros(n)
    _check(lib().bse_get_orbitals(ctx.h, n, _dev(out, "orbitals"), _dptr(e)))
    return out, e


def apply(ctx, X, Y=None):
    """bse_apply: Y = P_c M P_c X for X [n_b][n_val][n_pw] (CUDA float64)."""
    import torch
    if Y is None:
        Y = torch.empty_like(X)
    nb = X.shape[0] if X.dim() == 3 else 1
    _check(lib().bse_apply(ctx.h, nb, _dev(X, "X"), _dev(Y, "Y")))
    return Y


def _opts(tol=0.0, max_iter=0, block=0, max_subspace=0, x0=None, z0=None, use_learned=False,
          shifts=None, band_iters=None, two_level=False):
    o = SolverOpts()
    o.two_level = 1 if two_level else 0
    o.tol, o.max_iter, o.block, o.max_subspace = float(tol), int(max_iter), int(block), int(max_subspace)
    o.use_learned = 1 if use_learned else 0
    if shifts is not None:
        o.precond_shift_host = _dptr(shifts)
    if band_iters is not None:
        o.band_iters_host = band_iters.ctypes.data_as(C.POINTER(C.c_int32))
    if x0 is not None:
        o.x0_dev = _dev(x0, "x0").value
        o.n_x0 = x0.shape[0]
    if z0 is not None:
        o.z0_dev = _dev(z0, "z0").value
    return o


def _stats(s):
    return dict(iters=s.iters, applies=s.applies, resid=list(s.resid), t_ms=s.t_ms,
                applies_fp64=s.applies_fp64, learned=s.learned, fallback=s.fallback,
                t_u_ms=s.t_u_ms)


def davidson(ctx, n_states=1, *, tol=1e-8, max_iter=0, block=0, max_subspace=0, x0=None,
             use_learned=False, shifts=None, two_level=False, check=True):
    import torch
    info = get_info(ctx)
    X = torch.empty((n_states, info["n_val"], info["n_pw"]), dtype=torch.float64, device="cuda")
    w = np.zeros(n_states)
    sh = None if shifts is None else _f64(shifts)
    o = _opts(tol, max_iter, block, max_subspace, x0=x0, use_learned=use_learned, shifts=sh,
              two_level=two_level)
    s = SolverStats()
    rc = lib().bse_davidson(ctx.h, n_states, C.byref(o), _dptr(w), _dev(X, "X"), C.byref(s))
    if check:
        _check(rc)
    return w, X, dict(_stats(s), rc=rc)


def apply_coupling(ctx, X, Y=None):
    """bse_apply_coupling: Y = P_c (s K2e - K2d) P_c X (beyond the TDA)."""
    import torch
    Y = torch.empty_like(X) if Y is None else Y
    nb = X.shape[0] if X.dim() == 3 else 1
    _check(lib().bse_apply_coupling(ctx.h, nb, _dev(X, "X"), _dev(Y, "Y")))
    return Y


def full_bse(ctx, n_states=1, *, tol=1e-8, max_iter=0, block=0, max_subspace=0):
    """bse_full_bse: lowest roots beyond the TDA; returns (omega, X, Y, stats)."""
    import torch
    info = get_info(ctx)
    X = torch.empty((n_states, info["n_val"], info["n_pw"]), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    om = np.zeros(n_states)
    o = _opts(tol=tol, max_iter=max_iter, block=block, max_subspace=max_subspace)
    s = SolverStats()
    _check(lib().bse_full_bse(ctx.h, n_states, C.byref(o), _dptr(om), _dev(X, "X"), _dev(Y, "Y"),
                              C.byref(s)))
    return om, X, Y, _stats(s)


def u_vector(ctx, Xs):
    import torch
    U = torch.empty_like(Xs)
    _check(lib().bse_u_vector(ctx.h, _dev(Xs, "Xs"), _dev(U, "U")))
    return U


def zvector_solve(ctx, Xs, *, tol=1e-8, max_iter=0, z0=None, use_learned=False, shifts=None,
                  band_iters=False, two_level=False, check=True):
    """bse_zvector_solve.  shifts: per-band preconditioner shifts (host);
    band_iters=True adds the per-band iteration counts to the stats."""
    import torch
    Z = torch.empty_like(Xs)
    sh = None if shifts is None else _f64(shifts)
    bi = np.zeros(Xs.shape[0], dtype=np.int32) if band_iters else None
    o = _opts(tol, max_iter, z0=z0, use_learned=use_learned, shifts=sh, band_iters=bi,
              two_level=two_level)
    s = SolverStats()
    rc = lib().bse_zvector_solve(ctx.h, _dev(Xs, "Xs"), C.byref(o), _dev(Z, "Z"), C.byref(s))
    if check:
        _check(rc)
    st = dict(_stats(s), rc=rc)
    if bi is not None:
        st["band_iters"] = bi
    return Z, st


def forces(ctx, Xs, Z, n_sites):
    out = np.zeros((max(n_sites, 1), 3))
    _check(lib().bse_forces(ctx.h, _dev(Xs, "Xs"), _dev(Z, "Z"), _dptr(out)))
    return out[:n_sites]


def forces_noalloc(ctx, Xs, Z, out):
    """bse_forces_noalloc: d omega/d R into the caller's device tensor out
    [n_sites][3] (float64, contiguous); stream ordered, no allocation."""
    _check(lib().bse_forces_noalloc(ctx.h, _dev(Xs, "Xs"), _dev(Z, "Z"),
                                    _dev(out, "out") if out.numel() else None))
    return out


def ground_state_forces(ctx, n_sites):
    """bse_ground_state_forces: d(sum_v eps_v)/dR [n_sites][3] (Hellmann-Feynman)."""
    out = np.zeros((max(n_sites, 1), 3))
    _check(lib().bse_ground_state_forces(ctx.h, _dptr(out)))
    return out[:n_sites]


class Mlp:
    """The learned preconditioner's network (bse_mlp_*): owns the handle."""

    def __init__(self, n_in=LEARN_NFEAT, n_out=LEARN_NOUT, seed=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(lib().bse_mlp_create(int(n_in), int(n_out), int(seed), C.c_void_p(stream),
                                    C.byref(h)))
        self.h, self.n_in, self.n_out = h, int(n_in), int(n_out)
        n = C.c_int64()
        _check(lib().bse_mlp_n_params(self.h, C.byref(n)))
        self.n_params = int(n.value)

    def free(self):
        if self.h is not None and self.h.value and _lib is not None:
            _lib.bse_mlp_free(self.h)
            self.h = C.c_void_p(None)

    def __del__(self):
        self.free()

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.n_params
        _check(lib().bse_mlp_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().bse_mlp_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def set_norm(self, mu_x, s_x, mu_y, s_y):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (mu_x, s_x, mu_y, s_y)]
        _check(lib().bse_mlp_set_norm(self.h, *[a.ctypes.data_as(C.POINTER(C.c_float))
                                                for a in arrs]))

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        _check(lib().bse_mlp_forward(self.h, x.shape[0], _fdev(x, "x"), _fdev(y, "y")))
        return y

    def train_step(self, x, t, w=None, lr=1e-3, want_grad=False):
        import torch
        loss = C.c_float()
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda") if want_grad else None
        _check(lib().bse_mlp_train_step(self.h, x.shape[0], _fdev(x, "x"), _fdev(t, "t"),
                                        None if w is None else _fdev(w, "w"), float(lr),
                                        C.byref(loss), None if g is None else _fdev(g, "g")))
        return (float(loss.value), g) if want_grad else float(loss.value)


def _fdev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def set_graphs(ctx, on=True):
    """bse_set_graphs: replay captured HIP graphs for the block applies."""
    _check(lib().bse_set_graphs(ctx.h, 1 if on else 0))


def set_learned(ctx, mlp):
    """bse_set_learned: attach (or, with None, detach) a network."""
    _check(lib().bse_set_learned(ctx.h, None if mlp is None else mlp.h))
    ctx._learned = mlp  # keep it alive while attached


def learned_features(ctx, Xs, Zref=None, two_level=False):
    """bse_learned_features: features [n_val][8] and, with Zref, gamma* [n_val]."""
    nv = Xs.shape[0]
    f = np.zeros((nv, LEARN_NFEAT), dtype=np.float32)
    g = np.zeros(nv) if Zref is not None else None
    _check(lib().bse_learned_features(ctx.h, _dev(Xs, "Xs"),
                                      None if Zref is None else _dev(Zref, "Zref"),
                                      1 if two_level else 0,
                                      f.ctypes.data_as(C.POINTER(C.c_float)),
                                      None if g is None else _dptr(g)))
    return (f, g) if Zref is not None else f


def set_precision(ctx, precision):
    """bse_set_precision: FP64 or MIXED for the applies of a MIXED context."""
    _check(lib().bse_set_precision(ctx.h, int(precision)))


def warm_up():
    """bse_warm_up: HIP runtime start and device-code load, once per process."""
    _check(lib().bse_warm_up())


def set_profiling(ctx, on=True):
    _check(lib().bse_set_profiling(ctx.h, 1 if on else 0))


def phase_times(ctx, reset=False):
    p = PhaseTimes()
    _check(lib().bse_get_phase_times(ctx.h, C.byref(p), 1 if reset else 0))
    return {p.name[i].decode(): (p.ms[i], p.count[i]) for i in range(p.n_phase)}


def free(ctx):
    ctx.free()


def memory_cache(on=True):
    """bse_memory_cache: keep freed contexts' device memory for later ones."""
    _check(lib().bse_memory_cache(1 if on else 0))
