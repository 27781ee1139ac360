"""Python binding of librp (include/rp.h): argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch provides device
memory and the stream.  Importing this module does not need a GPU; calling a
device entry point does, and fails loudly if the library is not built.
"""
import ctypes
import os

import numpy as np

from .workloads import GAMMA_E, SpinSystem

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librp.so")

RP_OK, RP_EINVAL, RP_ENOMEM, RP_EDEVICE, RP_ENOTCONV, RP_ENOTIMPL = 0, -1, -2, -3, -4, -5


class RpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librp error {code}: {msg}")
        self.code = code


class _System(ctypes.Structure):
    _fields_ = [("n_nuc", ctypes.c_int32 * 2), ("two_I", ctypes.POINTER(ctypes.c_int32)),
                ("a_mT", ctypes.POINTER(ctypes.c_double)), ("J_mT", ctypes.c_double),
                ("kS", ctypes.c_double), ("kT", ctypes.c_double), ("T_us", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("init_mode", ctypes.c_int32), ("tol", ctypes.c_double),
                ("rdt", ctypes.c_double), ("r_scale", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("krylov_dim", ctypes.c_int32), ("max_growth", ctypes.c_double),
                ("ps_t_len", ctypes.c_int64)]


_lib = None

EXPORTS = ["rp_sample", "rp_propagate", "rp_yield", "rp_strerror", "rp_last_error", "rp_bessel_j",
           "rp_plan_field", "rp_profile_last", "rp_mlp_param_count", "rp_mlp_workspace_floats",
           "rp_mlp_features", "rp_mlp_forward", "rp_mlp_train_step", "rp_cv_beta", "rp_combine",
           "rp_design_size", "rp_group_mean", "rp_propagate_static", "rp_probe_stream",
           "rp_mlp_standardize", "rp_mlp_loss"]
RP_FLAG_PROFILE = 1
RP_FLAG_TILED = 2
RP_FLAG_XCD_LOCAL = 4
RP_FLAG_XCD_SPREAD = 8
RP_FLAG_NO_GRAPH = 16
RP_FLAG_ARNOLDI = 32
RP_FLAG_TERM_SCALAR = 64
RP_FLAG_AXES_HIGH_FIRST = 128


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64)
        sp = ctypes.POINTER(_System)
        op = ctypes.POINTER(_Opts)
        L.rp_sample.argtypes = [sp, u64, u32, u64, i64, i32, vp, vp]
        L.rp_propagate.argtypes = [sp, i32, dp, i32, vp, i64, op, vp, vp, vp]
        L.rp_propagate_static.argtypes = [sp, i32, dp, i32, vp, i64, op, vp, vp, vp]
        L.rp_yield.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp]
        L.rp_mlp_param_count.argtypes = [i32, i32, i32]
        L.rp_mlp_param_count.restype = i64
        L.rp_mlp_workspace_floats.argtypes = [i32, i32, i32, i64]
        L.rp_mlp_workspace_floats.restype = i64
        L.rp_mlp_features.argtypes = [vp, i64, i32, vp, i32, i32, i32, u64, vp, vp]
        L.rp_cv_beta.argtypes = [vp, vp, i32, i64, vp, vp]
        L.rp_combine.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp]
        L.rp_design_size.argtypes = [i32, i32]
        L.rp_design_size.restype = i64
        L.rp_group_mean.argtypes = [vp, i32, i64, i64, vp, vp]
        L.rp_mlp_forward.argtypes = [i32, i32, i32, vp, vp, i64, vp, vp, vp]
        L.rp_mlp_standardize.argtypes = [vp, i32, i64, i64, vp, vp]
        L.rp_mlp_standardize.restype = ctypes.c_int
        L.rp_mlp_loss.argtypes = [i32, i32, i32, vp, vp, vp, i64, vp, vp, vp]
        L.rp_mlp_loss.restype = ctypes.c_int
        L.rp_mlp_train_step.argtypes = [i32, i32, i32, vp, vp, vp, i64, vp, vp, i64, ctypes.c_float, vp, vp,
                                        vp, vp]
        L.rp_strerror.argtypes = [ctypes.c_int]
        L.rp_strerror.restype = ctypes.c_char_p
        L.rp_last_error.restype = ctypes.c_char_p
        L.rp_bessel_j.argtypes = [ctypes.c_double, i32, dp]
        L.rp_plan_field.argtypes = [sp, ctypes.c_double, op, dp, dp, dp]
        L.rp_profile_last.argtypes = [dp, i32]
        L.rp_probe_stream.argtypes = [i32, vp, vp, vp, i64, i32, dp, vp]
        L.rp_probe_stream.restype = ctypes.c_int
        for f in ("rp_sample", "rp_propagate", "rp_propagate_static", "rp_yield", "rp_bessel_j", "rp_plan_field", "rp_profile_last",
                  "rp_mlp_features", "rp_mlp_forward", "rp_mlp_train_step", "rp_cv_beta", "rp_combine",
                  "rp_group_mean"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code != RP_OK:
        L = lib()
        raise RpError(code, f"{L.rp_strerror(code).decode()}: {L.rp_last_error().decode()}")


class _CSystem:
    """Keeps the host arrays of one rp_system alive while a call runs."""

    def __init__(self, s: SpinSystem):
        self.two_I = np.ascontiguousarray(s.two_I if s.N else [0], np.int32)
        self.a = np.ascontiguousarray(s.a_mT if s.N else [0.0], np.float64)
        self.c = _System()
        self.c.n_nuc[0], self.c.n_nuc[1] = s.n1, s.n2
        self.c.two_I = self.two_I.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.c.a_mT = self.a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.c.J_mT, self.c.kS, self.c.kT, self.c.T_us = s.J_mT, s.kS, s.kT, s.T_us
        self.c.gamma = s.gamma if s.gamma else GAMMA_E


def _opts(precision=64, init_mode=0, tol=0.0, rdt=0.0, r_scale=0.0, workspace_bytes=0, flags=0, max_growth=0.0,
          krylov_dim=0, ps_t_len=0):
    o = _Opts()
    o.precision, o.init_mode, o.tol, o.rdt, o.r_scale = precision, init_mode, tol, rdt, r_scale
    o.workspace_bytes, o.flags, o.krylov_dim, o.max_growth = workspace_bytes, flags, krylov_dim, max_growth
    o.ps_t_len = ps_t_len
    return o


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype):
    import torch
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor of dtype %s" % dtype)
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------- device entry points
def design_size(n_nuclei, basis_mode):
    """rp_design_size: samples per group of a sampler mode (1 for modes 0-2)."""
    r = lib().rp_design_size(n_nuclei, basis_mode)
    if r < 0:
        _check(int(r))
    return int(r)


def sample(system: SpinSystem, seed, M, first=0, stream_id=0, basis_mode=0, out=None):
    """rp_sample: [M][N][2] float64 CUDA tensor of directions (or basis digits); modes 3 and 4
    are the sign-flip designs (groups of design_size(N, mode) samples)."""
    import torch
    cs = _CSystem(system)
    if out is None:
        out = torch.empty((M, system.N, 2), dtype=torch.float64, device="cuda")
    _check(lib().rp_sample(ctypes.byref(cs.c), seed, stream_id, first, M, basis_mode,
                           _dev_ptr(out, torch.float64), _stream(torch)))
    return out


def propagate(systems, B_mT, angles, M, precision=64, init_mode=0, tol=0.0, rdt=0.0, r_scale=0.0,
              workspace_bytes=0, out=None, profile=False, tiled=False, xcd=None, graph=True, max_growth=0.0,
              arnoldi=False, krylov_dim=0, term_scalar=False, ps_t_len=0, static=False, axes_high_first=False):
    """rp_propagate: single-wavepacket yields [n_sys][nB][M] (float64 CUDA tensor).
    With ``static`` the call goes to rp_propagate_static (no device allocation inside the
    library: its static workspace area instead).

    ``systems`` is a SpinSystem or a list; ``B_mT`` is [n_sys][nB] (host);
    ``angles`` is the concatenation of the per-system [M][N][2] arrays (CUDA).
    With ``ps_t_len`` > 0 it returns (yields, singlet populations at the step starts
    [n_sys][nB][M][ps_t_len], NaN past a field's last step).
    """
    import torch
    if isinstance(systems, SpinSystem):
        systems = [systems]
    B = np.ascontiguousarray(np.atleast_2d(np.asarray(B_mT, np.float64)))
    if B.shape[0] != len(systems):
        raise ValueError("B_mT must have one row per system")
    nB = B.shape[1]
    cs = [_CSystem(s) for s in systems]
    arr = (_System * len(cs))(*[c.c for c in cs])
    if out is None:
        out = torch.empty((len(systems), nB, M), dtype=torch.float64, device="cuda")
    ang = _dev_ptr(angles, torch.float64) if angles is not None and angles.numel() else None
    flags = (RP_FLAG_PROFILE if profile else 0) | (RP_FLAG_TILED if tiled else 0)
    flags |= (0 if graph else RP_FLAG_NO_GRAPH) | (RP_FLAG_ARNOLDI if arnoldi else 0)
    flags |= RP_FLAG_TERM_SCALAR if term_scalar else 0
    flags |= RP_FLAG_AXES_HIGH_FIRST if axes_high_first else 0
    if xcd == "local":
        flags |= RP_FLAG_XCD_LOCAL
    elif xcd == "spread":
        flags |= RP_FLAG_XCD_SPREAD
    o = _opts(precision, init_mode, tol, rdt, r_scale, workspace_bytes, flags, max_growth, krylov_dim, ps_t_len)
    ps = torch.empty((len(systems), nB, M, ps_t_len), dtype=torch.float64, device="cuda") if ps_t_len > 0 else None
    fn = lib().rp_propagate_static if static else lib().rp_propagate
    _check(fn(arr, len(cs), B.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nB, ang, M, ctypes.byref(o),
              _dev_ptr(out, torch.float64), _dev_ptr(ps, torch.float64), _stream(torch)))
    return (out, ps) if ps is not None else out


def combine(mean_a, err_a, mean_b, err_b):
    """rp_combine: inverse-variance combination of two independent per-field estimates (CUDA float64 [nB])."""
    import torch
    nB = mean_a.numel()
    mean = torch.empty(nB, dtype=torch.float64, device="cuda")
    err = torch.empty(nB, dtype=torch.float64, device="cuda")
    _check(lib().rp_combine(_dev_ptr(mean_a.contiguous(), torch.float64), _dev_ptr(err_a.contiguous(), torch.float64),
                            _dev_ptr(mean_b.contiguous(), torch.float64), _dev_ptr(err_b.contiguous(), torch.float64),
                            nB, _dev_ptr(mean, torch.float64), _dev_ptr(err, torch.float64), _stream(torch)))
    return mean, err


def group_mean(phi, group):
    """rp_group_mean: means of consecutive groups of ``group`` samples of phi [..][M] (CUDA float64)."""
    import torch
    phi = phi.reshape(-1, phi.shape[-1]).contiguous()
    nB, M = phi.shape
    out = torch.empty((nB, M // max(group, 1)), dtype=torch.float64, device="cuda")
    _check(lib().rp_group_mean(_dev_ptr(phi, torch.float64), nB, M, group, _dev_ptr(out, torch.float64),
                               _stream(torch)))
    return out


def yield_stats(phi, cv_g=None, cv_mu=None, cv_beta=None, cv_mu_err=None):
    """rp_yield: per-field mean and standard error of phi [nB][M] (CUDA float64)."""
    import torch
    phi = phi.reshape(-1, phi.shape[-1]).contiguous()
    nB, M = phi.shape
    mean = torch.empty(nB, dtype=torch.float64, device="cuda")
    err = torch.empty(nB, dtype=torch.float64, device="cuda")
    g = _dev_ptr(cv_g.reshape(nB, M).contiguous(), torch.float64) if cv_g is not None else None
    mu = _dev_ptr(cv_mu.contiguous(), torch.float64) if cv_mu is not None else None
    be = _dev_ptr(cv_beta.contiguous(), torch.float64) if cv_beta is not None else None
    mv = _dev_ptr(cv_mu_err.contiguous(), torch.float64) if cv_mu_err is not None else None
    _check(lib().rp_yield(_dev_ptr(phi, torch.float64), nB, M, g, mu, be, mv, _dev_ptr(mean, torch.float64),
                          _dev_ptr(err, torch.float64), _stream(torch)))
    return mean, err


# ----------------------------------------------------------------------------- control-variate network
def mlp_param_count(n_in, width=256, depth=3):
    n = lib().rp_mlp_param_count(n_in, width, depth)
    if n < 0:
        raise ValueError("bad network shape")
    return n


def mlp_in_pad(n_in):
    return (n_in + 15) // 16 * 16


def mlp_workspace(n_in, width, depth, rows):
    import torch
    n = lib().rp_mlp_workspace_floats(n_in, width, depth, rows)
    return torch.empty(max(n, 1), dtype=torch.float32, device="cuda")


def mlp_features(angles, B_mT, n_in, layout=0, rot_seed=0):
    """rp_mlp_features: [nB*M][n_in_pad] float32 features (row layouts 0, 1, 2 of rp.h); a
    nonzero rot_seed rotates each row's directions about the field axis (augmentation)."""
    import torch
    B = torch.as_tensor(np.asarray(B_mT, np.float64).reshape(-1), device="cuda")
    nB = B.numel()
    N = angles.shape[1]
    M = angles.shape[0] // nB if layout == 2 else angles.shape[0]
    x = torch.empty((nB * M, mlp_in_pad(n_in)), dtype=torch.float32, device="cuda")
    _check(lib().rp_mlp_features(_dev_ptr(angles.contiguous(), torch.float64), M, N, _dev_ptr(B, torch.float64),
                                 nB, x.shape[1], int(layout), int(rot_seed), _dev_ptr(x, torch.float32),
                                 _stream(torch)))
    return x


def cv_beta(phi, g):
    """rp_cv_beta: per-field Cov(phi, g)/Var(g) for device float64 [nB][M] arrays."""
    import torch
    phi = phi.contiguous()
    g = g.contiguous()
    nB, M = phi.shape
    beta = torch.empty(nB, dtype=torch.float64, device="cuda")
    _check(lib().rp_cv_beta(_dev_ptr(phi, torch.float64), _dev_ptr(g, torch.float64), nB, M,
                            _dev_ptr(beta, torch.float64), _stream(torch)))
    return beta


def mlp_forward(params, x, n_in, width=256, depth=3, workspace=None):
    import torch
    rows = x.shape[0]
    y = torch.empty(rows, dtype=torch.float32, device="cuda")
    ws = workspace if workspace is not None else mlp_workspace(n_in, width, depth, rows)
    _check(lib().rp_mlp_forward(n_in, width, depth, _dev_ptr(params, torch.float32), _dev_ptr(x, torch.float32),
                                rows, _dev_ptr(y, torch.float32), _dev_ptr(ws, torch.float32), _stream(torch)))
    return y


def mlp_standardize(phi, nB, n_rows, n_fit):
    """rp_mlp_standardize: float32 CUDA targets [n_rows * nB] from float64 phi (row s*nB + b)."""
    import torch
    phi = phi.contiguous()
    t = torch.empty(n_rows * nB, dtype=torch.float32, device="cuda")
    _check(lib().rp_mlp_standardize(_dev_ptr(phi, torch.float64), nB, n_rows, n_fit, _dev_ptr(t, torch.float32),
                                    _stream(torch)))
    return t


def mlp_loss(params, x, target, n_in, width=256, depth=3, workspace=None):
    """rp_mlp_loss: mean squared error of the network on (x, target), as a CUDA float64 scalar."""
    import torch
    rows = x.shape[0]
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = workspace if workspace is not None else mlp_workspace(n_in, width, depth, rows)
    _check(lib().rp_mlp_loss(n_in, width, depth, _dev_ptr(params, torch.float32), _dev_ptr(x, torch.float32),
                             _dev_ptr(target.contiguous(), torch.float32), rows, _dev_ptr(out, torch.float64),
                             _dev_ptr(ws, torch.float32), _stream(torch)))
    return out


def mlp_train_step(params, adam_m, adam_v, step, x, target, n_in, width=256, depth=3, lr=1e-3,
                   grad_out=None, sq_err=None, workspace=None):
    import torch
    rows = x.shape[0]
    ws = workspace if workspace is not None else mlp_workspace(n_in, width, depth, rows)
    _check(lib().rp_mlp_train_step(n_in, width, depth, _dev_ptr(params, torch.float32),
                                   _dev_ptr(adam_m, torch.float32), _dev_ptr(adam_v, torch.float32), step,
                                   _dev_ptr(x, torch.float32), _dev_ptr(target, torch.float32), rows,
                                   float(lr), _dev_ptr(grad_out, torch.float32), _dev_ptr(sq_err, torch.float32),
                                   _dev_ptr(ws, torch.float32), _stream(torch)))


def probe_stream(bytes_, reps=10):
    """rp_probe_stream over fresh CUDA buffers of bytes_ bytes: GB/s of each streaming pattern,
    counting every byte read and written: {"copy": .., "read2_write1": .., "read": .., "write": ..}."""
    import torch
    n = bytes_ // 16 * 16
    bufs = [torch.ones(n // 4, dtype=torch.float32, device="cuda") for _ in range(3)]
    out = {}
    moved = {0: 2, 1: 3, 2: 1, 3: 1}
    for kind, name in ((0, "copy"), (1, "read2_write1"), (2, "read"), (3, "write")):
        ms = ctypes.c_double(0.0)
        _check(lib().rp_probe_stream(kind, _dev_ptr(bufs[0], torch.float32), _dev_ptr(bufs[1], torch.float32),
                                     _dev_ptr(bufs[2], torch.float32), n, reps, ctypes.byref(ms), _stream(torch)))
        out[name] = moved[kind] * n / (ms.value * 1e-3) / 1e9
    return out


def profile_last():
    """Timing totals of the last profiled rp_propagate call on this thread (see rp.h)."""
    out = np.zeros(8)
    lib().rp_profile_last(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 8)
    keys = ["term_ms", "term_launches", "elements", "bytes_per_element", "quad_ms", "quad_launches",
            "total_ms", "terms_per_step"]
    return dict(zip(keys, out.tolist()))


# ----------------------------------------------------------------------------- host-only helpers
def bessel_j(x, nmax):
    out = np.zeros(nmax + 1)
    _check(lib().rp_bessel_j(float(x), int(nmax), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def plan_field(system: SpinSystem, B_mT, precision=64, tol=0.0, rdt=0.0, r_scale=0.0, max_growth=0.0):
    """Chebyshev step plan of one field: dict with r, c, dt, n_steps, n_terms, rank, x, coef, ell."""
    cs = _CSystem(system)
    o = _opts(precision, 0, tol, rdt, r_scale, max_growth=max_growth)
    info = np.zeros(8)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().rp_plan_field(ctypes.byref(cs.c), float(B_mT), ctypes.byref(o), info.ctypes.data_as(dp),
                               None, None))
    nt, rk = int(info[5]), int(info[6])
    coef = np.zeros(2 * nt)
    ell = np.zeros(nt * rk)
    _check(lib().rp_plan_field(ctypes.byref(cs.c), float(B_mT), ctypes.byref(o), info.ctypes.data_as(dp),
                               coef.ctypes.data_as(dp), ell.ctypes.data_as(dp)))
    return dict(r=info[0], c=complex(info[1], info[2]), dt=info[3], n_steps=int(info[4]), n_terms=nt,
                rank=rk, x=info[7], coef=coef[0::2] + 1j * coef[1::2], ell=ell.reshape(nt, rk))
