"""Thin ctypes binding of libtdvp (include/tdvp.h).

Only argument marshalling happens here: torch tensors provide device memory
and the HIP stream, every step of the TDVP-PS path runs in the library's
kernels.  If the library is not built the import of any entry point raises;
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdvp.so")

FP64 = 0
FP32 = 1
BF16X3 = 2

HARTREE_PER_CM = 4.556335252767e-6   # 1 cm^-1 in hartree
AU_PER_FS = 41.341373335             # 1 fs in atomic units of time


class TdvpError(RuntimeError):
    pass


class _Mps(ctypes.Structure):
    _fields_ = [("n", c_int32), ("phys", POINTER(c_int32)), ("bond", POINTER(c_int32)),
                ("site", POINTER(c_void_p))]


class _Mpo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("phys", POINTER(c_int32)), ("bond", POINTER(c_int32)),
                ("site", POINTER(c_void_p)), ("energy_shift", c_double)]


class _Envs(ctypes.Structure):
    _fields_ = [("left", POINTER(c_void_p)), ("right", POINTER(c_void_p))]


EXPORTS = {
    "tdvp_create": (c_int, [POINTER(c_void_p), c_int, c_void_p, c_int]),
    "tdvp_destroy": (c_int, [c_void_p]),
    "tdvp_set_stream": (c_int, [c_void_p, c_void_p]),
    "tdvp_status_string": (ctypes.c_char_p, [c_int]),
    "tdvp_env_elem_bytes": (c_int, [c_void_p]),
    "tdvp_workspace_bytes": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_int, POINTER(c_size_t)]),
    "tdvp_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
    "tdvp_env_update": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int,
                                c_int, c_int, c_void_p]),
    "tdvp_heff_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                c_int, c_void_p, c_void_p]),
    "tdvp_lanczos_expm": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                  c_int, c_double, c_double, c_int, c_double, c_void_p, c_void_p,
                                  c_void_p]),
    "tdvp_lanczos_expm_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_int,
                                          c_int, c_int, c_double, c_double, c_int, c_double, c_void_p,
                                          c_void_p, c_void_p]),
    "tdvp_qr": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "tdvp_right_canonicalize": (c_int, [c_void_p, POINTER(_Mps)]),
    "tdvp_left_canonicalize": (c_int, [c_void_p, POINTER(_Mps)]),
    "tdvp_envs_build": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs)]),
    "tdvp_ps2_workspace_bytes": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_int, POINTER(c_size_t)]),
    "tdvp_svd_split": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "tdvp_ps2_step": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs), c_double, c_int,
                              c_int, c_double, c_void_p]),
    "tdvp_ps_step": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs), c_double, c_int,
                             c_int, c_double]),
    "tdvp_observe": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs), POINTER(c_int32),
                             c_int, c_void_p]),
    "tdvp_set_krylov_log": (c_int, [c_void_p, c_void_p, c_int]),
    "tdvp_set_graph": (c_int, [c_void_p, c_int]),
    "tdvp_set_fused": (c_int, [c_void_p, c_int]),
    "tdvp_set_stage3_split": (c_int, [c_void_p, c_int]),
    "tdvp_set_autotune": (c_int, [c_void_p, c_int]),
    "tdvp_profile_reps": (c_int, [c_void_p, c_int]),
    "tdvp_autotune_count": (c_int, [c_void_p, c_void_p]),
    "tdvp_ps_step_batched": (c_int, [c_void_p, c_int, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs),
                                     c_double, c_int, c_int, c_double]),
    "tdvp_observe_batched": (c_int, [c_void_p, c_int, POINTER(_Mps), POINTER(_Mpo), POINTER(_Envs),
                                     POINTER(c_int32), c_int, c_void_p]),
    "tdvp_profile": (c_int, [c_void_p, c_int]),
    "tdvp_profile_read": (c_int, [c_void_p, POINTER(c_double), POINTER(c_int64), POINTER(c_double),
                                  POINTER(c_double)]),
    "tdvp_workspace_bytes_grouped": (c_int, [c_void_p, c_int, POINTER(c_int32), POINTER(_Mps),
                                             POINTER(_Mpo), c_int, POINTER(c_size_t)]),
    "tdvp_ps_step_grouped": (c_int, [c_void_p, c_int, POINTER(c_int32), POINTER(_Mps), POINTER(_Mpo),
                                     POINTER(_Envs), c_double, c_int, c_int, c_double]),
    "tdvp_observe_grouped": (c_int, [c_void_p, c_int, POINTER(c_int32), POINTER(_Mps), POINTER(_Mpo),
                                     POINTER(_Envs), POINTER(c_int32), c_int, c_void_p]),
    "tdvp_mu_workspace_bytes": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), POINTER(c_size_t)]),
    "tdvp_mu_rhs": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_double, POINTER(c_void_p)]),
    "tdvp_mu_evolve": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_double, c_double, c_double,
                               c_double, c_int, POINTER(c_int64)]),
    "tdvp_mu_cmf_workspace_bytes": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_int,
                                            POINTER(c_size_t)]),
    "tdvp_mu_cmf_step": (c_int, [c_void_p, POINTER(_Mps), POINTER(_Mpo), c_double, c_double, c_double,
                                 c_double, c_int, c_int, c_double, POINTER(c_int64)]),
    "tdvp_holstein_mpo": (c_int, [c_int, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32), c_int,
                                  POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                  POINTER(c_double), POINTER(c_int32), POINTER(c_int64),
                                  POINTER(c_double)]),
}

_lib = None


def lib():
    """Load libtdvp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TdvpError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, what):
    if status != 0:
        msg = lib().tdvp_status_string(status).decode()
        raise TdvpError(f"{what}: {msg} (status {status})")


def _ptr(t):
    return c_void_p(t.data_ptr())


def _i32(a):
    return (c_int32 * len(a))(*[int(v) for v in a])


# ---------------------------------------------------------------- host MPO

def holstein_mpo(kind, owner, phys, eps, J, w, g):
    """Frenkel-Holstein MPO tensors (host numpy complex128), built by the library."""
    n = len(kind)
    n_e = int(np.asarray(eps).size)
    bond = (c_int32 * (n + 1))()
    total = c_int64(0)
    k, o, p = _i32(kind), _i32(owner), _i32(phys)
    epsa = np.ascontiguousarray(eps, dtype=np.float64)
    Ja = np.ascontiguousarray(J, dtype=np.float64).reshape(-1)
    wa = np.ascontiguousarray(w, dtype=np.float64)
    ga = np.ascontiguousarray(g, dtype=np.float64)
    dp = POINTER(c_double)
    _check(lib().tdvp_holstein_mpo(n, k, o, p, n_e, epsa.ctypes.data_as(dp), Ja.ctypes.data_as(dp),
                                   wa.ctypes.data_as(dp), ga.ctypes.data_as(dp), bond,
                                   ctypes.byref(total), None), "tdvp_holstein_mpo(query)")
    out = np.zeros(2 * total.value, dtype=np.float64)
    _check(lib().tdvp_holstein_mpo(n, k, o, p, n_e, epsa.ctypes.data_as(dp), Ja.ctypes.data_as(dp),
                                   wa.ctypes.data_as(dp), ga.ctypes.data_as(dp), bond,
                                   ctypes.byref(total), out.ctypes.data_as(dp)), "tdvp_holstein_mpo")
    cpx = out.view(np.complex128)
    Ws = []
    off = 0
    for i in range(n):
        shape = (bond[i], phys[i], phys[i], bond[i + 1])
        size = int(np.prod(shape))
        Ws.append(cpx[off:off + size].reshape(shape).copy())
        off += size
    return Ws, [bond[i] for i in range(n + 1)]


def fmo_model(params, sites):
    """MPO inputs of an FMO-like chain: energies in hartree, constant offset removed.

    Returns (Ws, mpo_bond, energy_shift) where H' = H - energy_shift on the
    one-exciton sector (shift = mean site energy + zero-point energy).
    """
    E = np.asarray(params.E) * HARTREE_PER_CM
    Ebar = float(np.mean(E))
    eps = E - Ebar
    J = np.asarray(params.J) * HARTREE_PER_CM
    kind, owner, phys, w, g = [], [], [], [], []
    for s in sites:
        kind.append(0 if s[0] == "el" else 1)
        owner.append(s[1])
        phys.append(s[3])
        if s[0] == "el":
            w.append(0.0)
            g.append(0.0)
        else:
            w.append(params.omega[s[1], s[2]] * HARTREE_PER_CM)
            g.append(np.sqrt(params.S[s[1], s[2]]))
    shift = Ebar + 0.5 * float(np.sum(w))
    Ws, bond = holstein_mpo(kind, owner, phys, eps, J, w, g)
    return Ws, bond, shift


# ---------------------------------------------------------------- device objects

class Context:
    """A libtdvp context bound to a torch CUDA (HIP) stream, plus its workspace."""

    def __init__(self, device=0, precision=FP64, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = c_void_p()
        _check(lib().tdvp_create(ctypes.byref(h), device, c_void_p(stream.cuda_stream), precision),
               "tdvp_create")
        self.h = h
        self.ws = None

    @property
    def env_dtype(self):
        return self.torch.complex128 if self.precision == FP64 else self.torch.complex64

    def reserve(self, nbytes):
        """Make sure the workspace holds at least nbytes (a torch uint8 buffer)."""
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = self.torch.empty(int(nbytes) + 256, dtype=self.torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            _check(lib().tdvp_set_workspace(self.h, c_void_p(base + off), int(nbytes)),
                   "tdvp_set_workspace")

    def close(self):
        if self.h:
            lib().tdvp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceMps:
    """MPS site tensors (complex128 torch tensors on the GPU) with a C descriptor."""

    def __init__(self, tensors, device):
        import torch
        self.t = [torch.as_tensor(np.ascontiguousarray(A), dtype=torch.complex128).to(device)
                  for A in tensors]
        self.phys = [A.shape[1] for A in self.t]
        self.bond = [self.t[0].shape[0]] + [A.shape[2] for A in self.t]
        self._phys = _i32(self.phys)
        self._bond = _i32(self.bond)
        self._site = (c_void_p * len(self.t))(*[A.data_ptr() for A in self.t])
        self.desc = _Mps(len(self.t), self._phys, self._bond, self._site)

    def numpy(self):
        return [A.cpu().numpy() for A in self.t]


class DeviceMpo:
    def __init__(self, Ws, bond, shift, device):
        import torch
        self.t = [torch.as_tensor(np.ascontiguousarray(W), dtype=torch.complex128).to(device) for W in Ws]
        self.phys = [W.shape[1] for W in self.t]
        self.bond = list(bond)
        self.shift = float(shift)
        self._phys = _i32(self.phys)
        self._bond = _i32(self.bond)
        self._site = (c_void_p * len(self.t))(*[W.data_ptr() for W in self.t])
        self.desc = _Mpo(len(self.t), self._phys, self._bond, self._site, self.shift)


class DeviceEnvs:
    def __init__(self, mps_bond, mpo_bond, dtype, device):
        import torch
        n = len(mps_bond) - 1
        self.left = [torch.zeros((mps_bond[b], mpo_bond[b], mps_bond[b]), dtype=dtype, device=device)
                     for b in range(n + 1)]
        self.right = [torch.zeros((mps_bond[b], mpo_bond[b], mps_bond[b]), dtype=dtype, device=device)
                      for b in range(n + 1)]
        self._l = (c_void_p * (n + 1))(*[t.data_ptr() for t in self.left])
        self._r = (c_void_p * (n + 1))(*[t.data_ptr() for t in self.right])
        self.desc = _Envs(self._l, self._r)


# ---------------------------------------------------------------- entry points

def workspace_bytes(ctx, mps, mpo, kmax):
    b = c_size_t(0)
    _check(lib().tdvp_workspace_bytes(ctx.h, ctypes.byref(mps.desc),
                                      ctypes.byref(mpo.desc) if mpo is not None else None,
                                      kmax, ctypes.byref(b)), "tdvp_workspace_bytes")
    return b.value


def env_update(ctx, direction, env_in, A, W, Ml, d, Mr, Wl, Wr, env_out):
    _check(lib().tdvp_env_update(ctx.h, direction, _ptr(env_in), _ptr(A), _ptr(W), Ml, d, Mr, Wl, Wr,
                                 _ptr(env_out)), "tdvp_env_update")


def heff_apply(ctx, Lenv, W, Renv, Ml, d, Mr, Wl, Wr, x, y):
    _check(lib().tdvp_heff_apply(ctx.h, _ptr(Lenv), _ptr(W) if W is not None else None, _ptr(Renv),
                                 Ml, d, Mr, Wl, Wr, _ptr(x), _ptr(y)), "tdvp_heff_apply")


def lanczos_expm(ctx, Lenv, W, Renv, Ml, d, Mr, Wl, Wr, z, kmax, tol, x, y, k_used=None):
    _check(lib().tdvp_lanczos_expm(ctx.h, _ptr(Lenv), _ptr(W) if W is not None else None, _ptr(Renv),
                                   Ml, d, Mr, Wl, Wr, float(np.real(z)), float(np.imag(z)), kmax,
                                   float(tol), _ptr(x), _ptr(y),
                                   _ptr(k_used) if k_used is not None else None), "tdvp_lanczos_expm")


def lanczos_expm_noalloc(ctx, Lenv, W, Renv, Ml, d, Mr, Wl, Wr, z, kmax, tol, x, y, k_used=None):
    _check(lib().tdvp_lanczos_expm_noalloc(ctx.h, _ptr(Lenv), _ptr(W) if W is not None else None,
                                           _ptr(Renv), Ml, d, Mr, Wl, Wr, float(np.real(z)),
                                           float(np.imag(z)), kmax, float(tol), _ptr(x), _ptr(y),
                                           _ptr(k_used) if k_used is not None else None),
           "tdvp_lanczos_expm_noalloc")


def qr(ctx, A, m, n, Q, R):
    _check(lib().tdvp_qr(ctx.h, _ptr(A), m, n, _ptr(Q), _ptr(R)), "tdvp_qr")


def right_canonicalize(ctx, mps):
    _check(lib().tdvp_right_canonicalize(ctx.h, ctypes.byref(mps.desc)), "tdvp_right_canonicalize")


def left_canonicalize(ctx, mps):
    _check(lib().tdvp_left_canonicalize(ctx.h, ctypes.byref(mps.desc)), "tdvp_left_canonicalize")


def envs_build(ctx, mps, mpo, envs):
    _check(lib().tdvp_envs_build(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc),
                                 ctypes.byref(envs.desc)), "tdvp_envs_build")


def set_graph(ctx, enable):
    _check(lib().tdvp_set_graph(ctx.h, 1 if enable else 0), "tdvp_set_graph")


def set_fused(ctx, enable):
    _check(lib().tdvp_set_fused(ctx.h, 1 if enable else 0), "tdvp_set_fused")


def set_stage3_split(ctx, per_channel):
    _check(lib().tdvp_set_stage3_split(ctx.h, 1 if per_channel else 0), "tdvp_set_stage3_split")


def set_autotune(ctx, enable):
    _check(lib().tdvp_set_autotune(ctx.h, 1 if enable else 0), "tdvp_set_autotune")


def autotune_count(ctx):
    n = ctypes.c_int32(0)
    _check(lib().tdvp_autotune_count(ctx.h, ctypes.byref(n)), "tdvp_autotune_count")
    return int(n.value)


def ps_step(ctx, mps, mpo, envs, dt, nsteps=1, kmax=20, tol=0.0):
    _check(lib().tdvp_ps_step(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc),
                              ctypes.byref(envs.desc), float(dt), int(nsteps), int(kmax), float(tol)),
           "tdvp_ps_step")


def ps2_workspace_bytes(ctx, mps, mpo, kmax=20):
    b = c_size_t(0)
    _check(lib().tdvp_ps2_workspace_bytes(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc), int(kmax),
                                          ctypes.byref(b)), "tdvp_ps2_workspace_bytes")
    return b.value


def svd_split(ctx, X, m, n, keep, mode, A, B, discarded=None):
    _check(lib().tdvp_svd_split(ctx.h, _ptr(X), int(m), int(n), int(keep), int(mode), _ptr(A), _ptr(B),
                                None if discarded is None else _ptr(discarded)), "tdvp_svd_split")


def ps2_step(ctx, mps, mpo, envs, dt, nsteps=1, kmax=20, tol=0.0, discarded=None):
    """Two-site TDVP-PS steps; discarded: a device float64 tensor the dropped weight is added to."""
    _check(lib().tdvp_ps2_step(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc), ctypes.byref(envs.desc),
                               float(dt), int(nsteps), int(kmax), float(tol),
                               None if discarded is None else _ptr(discarded)), "tdvp_ps2_step")


def observe(ctx, mps, mpo, envs, el_sites, out):
    arr = _i32(el_sites)
    _check(lib().tdvp_observe(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc),
                              ctypes.byref(envs.desc), arr, len(el_sites), _ptr(out)), "tdvp_observe")


PROF_GEMM, PROF_WAPPLY, PROF_LZ_DOTS, PROF_LZ_UPDATE, PROF_LZ_ENDS, PROF_QR = 1, 2, 3, 4, 5, 6
PROF_LZ_FUSED = 7
PROF_GEMM_HEFF = 8
PROF_CLASSES = {"gemm": PROF_GEMM, "gemm_heff": PROF_GEMM_HEFF, "wapply": PROF_WAPPLY, "lz_dots": PROF_LZ_DOTS,
                "lz_update": PROF_LZ_UPDATE, "lz_ends": PROF_LZ_ENDS, "qr": PROF_QR,
                "lz_fused": PROF_LZ_FUSED}


def set_krylov_log(ctx, buf):
    """Log the Krylov dimension of every solve of the next ps_step calls into buf (int32)."""
    if buf is None:
        _check(lib().tdvp_set_krylov_log(ctx.h, None, 0), "tdvp_set_krylov_log")
    else:
        _check(lib().tdvp_set_krylov_log(ctx.h, _ptr(buf), buf.numel()), "tdvp_set_krylov_log")


def profile(ctx, kernel_class):
    _check(lib().tdvp_profile(ctx.h, kernel_class), "tdvp_profile")


def profile_reps(ctx, reps):
    _check(lib().tdvp_profile_reps(ctx.h, reps), "tdvp_profile_reps")


def profile_read(ctx):
    """(total ms, launches, algorithmic FLOP, algorithmic bytes) of the profiled launches."""
    ms, n, f, b = c_double(), c_int64(), c_double(), c_double()
    _check(lib().tdvp_profile_read(ctx.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(f),
                                   ctypes.byref(b)), "tdvp_profile_read")
    return ms.value, n.value, f.value, b.value


# ---------------------------------------------------------------- a whole run

class PsRun:
    """An FMO-like chain evolved with TDVP-PS on one GPU.

    ``raw_mps`` are the (non-canonical) initial site tensors; they are
    right-canonicalised and normalised on the device, the right environments
    built, and every later step runs through tdvp_ps_step (two_site=True:
    tdvp_ps2_step, FP64; the weight its SVDs drop accumulates in
    ``discarded``).  The run owns a
    HIP stream of its own (a captured step graph needs a non-NULL stream);
    every tensor of the run is created on that stream.
    """

    def __init__(self, params, sites, raw_mps, device=0, precision=FP64, kmax=20, tol=0.0,
                 graph=True, fused=True, autotune=False, stage3_split=False, two_site=False):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = Context(device, precision, stream=self.stream)
        dev = self.ctx.device
        self.sites = sites
        self.n_e = params.n_e
        with torch.cuda.stream(self.stream):
            Ws, wbond, shift = fmo_model(params, sites)
            self.mpo = DeviceMpo(Ws, wbond, shift, dev)
            self.mps = DeviceMps(raw_mps, dev)
            self.envs = DeviceEnvs(self.mps.bond, wbond, self.ctx.env_dtype, dev)
            self.kmax = kmax
            self.tol = tol
            ws = workspace_bytes(self.ctx, self.mps, self.mpo, kmax)
            self.two_site = two_site
            if two_site:
                ws = max(ws, ps2_workspace_bytes(self.ctx, self.mps, self.mpo, kmax))
                self.discarded = torch.zeros(1, dtype=torch.float64, device=dev)
            self.ctx.reserve(ws)
            self.el_sites = [0] * params.n_e
            for i, s in enumerate(sites):
                if s[0] == "el":
                    self.el_sites[s[1]] = i
            self.obs = torch.zeros(2 + params.n_e, dtype=torch.float64, device=dev)
        self.stream.synchronize()
        set_graph(self.ctx, graph)
        set_fused(self.ctx, fused)
        set_stage3_split(self.ctx, stage3_split)
        set_autotune(self.ctx, autotune)
        right_canonicalize(self.ctx, self.mps)
        envs_build(self.ctx, self.mps, self.mpo, self.envs)

    def step(self, dt_au, nsteps=1):
        if self.two_site:
            ps2_step(self.ctx, self.mps, self.mpo, self.envs, dt_au, nsteps, self.kmax, self.tol,
                     self.discarded)
        else:
            ps_step(self.ctx, self.mps, self.mpo, self.envs, dt_au, nsteps, self.kmax, self.tol)

    def observe(self, out=None):
        """Device tensor [norm^2, energy, populations...] (enqueued on the run's stream)."""
        out = self.obs if out is None else out
        observe(self.ctx, self.mps, self.mpo, self.envs, self.el_sites, out)
        return out

    def observe_host(self):
        out = self.observe()
        self.stream.synchronize()
        return out.cpu().numpy().copy()

    def synchronize(self):
        self.stream.synchronize()

    def mps_numpy(self):
        self.stream.synchronize()
        return self.mps.numpy()


# ---------------------------------------------------------------- TDVP-MU

def mu_workspace_bytes(ctx, mps, mpo):
    b = c_size_t(0)
    _check(lib().tdvp_mu_workspace_bytes(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc),
                                         ctypes.byref(b)), "tdvp_mu_workspace_bytes")
    return b.value


def mu_rhs(ctx, mps, mpo, eps, out_tensors):
    tab = (c_void_p * len(out_tensors))(*[t.data_ptr() for t in out_tensors])
    _check(lib().tdvp_mu_rhs(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc), float(eps), tab),
           "tdvp_mu_rhs")


def mu_evolve(ctx, mps, mpo, t_final, eps=1e-10, rtol=1e-5, atol=1e-8, max_steps=100000):
    """Integrate TDVP-MU in place; returns (accepted, rejected, rhs evaluations)."""
    st = (c_int64 * 3)()
    _check(lib().tdvp_mu_evolve(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc), float(t_final),
                                float(eps), float(rtol), float(atol), int(max_steps), st),
           "tdvp_mu_evolve")
    return tuple(int(v) for v in st)


def mu_cmf_workspace_bytes(ctx, mps, mpo, kmax=20):
    b = c_size_t(0)
    _check(lib().tdvp_mu_cmf_workspace_bytes(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc),
                                             int(kmax), ctypes.byref(b)), "tdvp_mu_cmf_workspace_bytes")
    return b.value


def mu_cmf_step(ctx, mps, mpo, tau, eps=1e-10, rtol=1e-10, atol=1e-12, max_steps=100000, kmax=20,
                tol=0.0):
    """One second-order constant-mean-field step in place; returns (accepted,
    rejected, site right-hand-side evaluations) summed over its two solves."""
    st = (c_int64 * 3)()
    _check(lib().tdvp_mu_cmf_step(ctx.h, ctypes.byref(mps.desc), ctypes.byref(mpo.desc), float(tau),
                                  float(eps), float(rtol), float(atol), int(max_steps), int(kmax),
                                  float(tol), st), "tdvp_mu_cmf_step")
    return tuple(int(v) for v in st)


class MuRun:
    """A chain evolved with TDVP-MU on one GPU from a LEFT-canonical MPS
    given as host arrays (canonicalize=True: any MPS, left-canonicalised
    on the device).  Own stream, FP64."""

    def __init__(self, params, sites, left_canonical_mps, device=0, canonicalize=False):
        import torch
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = Context(device, FP64, stream=self.stream)
        dev = self.ctx.device
        with torch.cuda.stream(self.stream):
            Ws, wbond, shift = fmo_model(params, sites)
            self.mpo = DeviceMpo(Ws, wbond, shift, dev)
            self.mps = DeviceMps(left_canonical_mps, dev)
            self.ctx.reserve(mu_workspace_bytes(self.ctx, self.mps, self.mpo))
            if canonicalize:
                left_canonicalize(self.ctx, self.mps)
        self.stream.synchronize()

    def rhs(self, eps=1e-10):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            out = [torch.empty_like(t) for t in self.mps.t]
        mu_rhs(self.ctx, self.mps, self.mpo, eps, out)
        self.stream.synchronize()
        return [t.cpu().numpy() for t in out]

    def evolve(self, t_final, eps=1e-10, rtol=1e-5, atol=1e-8, max_steps=100000):
        st = mu_evolve(self.ctx, self.mps, self.mpo, t_final, eps, rtol, atol, max_steps)
        self.stream.synchronize()
        return st

    def cmf_step(self, tau, nsteps=1, eps=1e-10, rtol=1e-10, atol=1e-12, max_steps=100000, kmax=20, tol=0.0):
        """nsteps constant-mean-field steps; returns the summed statistics."""
        self.ctx.reserve(mu_cmf_workspace_bytes(self.ctx, self.mps, self.mpo, kmax))
        tot = [0, 0, 0]
        for _ in range(nsteps):
            st = mu_cmf_step(self.ctx, self.mps, self.mpo, tau, eps, rtol, atol, max_steps, kmax, tol)
            tot = [a + b for a, b in zip(tot, st)]
        self.stream.synchronize()
        return tuple(tot)

    def mps_numpy(self):
        self.stream.synchronize()
        return self.mps.numpy()


# ---------------------------------------------------------------- ensembles

def ps_step_batched(ctx, descs, dt, nsteps=1, kmax=20, tol=0.0):
    mps_arr, mpo_arr, env_arr = descs
    _check(lib().tdvp_ps_step_batched(ctx.h, len(mps_arr), mps_arr, mpo_arr, env_arr, float(dt),
                                      int(nsteps), int(kmax), float(tol)), "tdvp_ps_step_batched")


def observe_batched(ctx, descs, el_sites, out):
    mps_arr, mpo_arr, env_arr = descs
    arr = _i32(el_sites)
    _check(lib().tdvp_observe_batched(ctx.h, len(mps_arr), mps_arr, mpo_arr, env_arr, arr,
                                      len(el_sites), _ptr(out)), "tdvp_observe_batched")


class PsEnsemble:
    """Independent chains of identical shape evolved together (one launch per kernel).

    Each site tensor of the ensemble is one (nb, ...) device array, so every
    instance sits at a constant stride from instance 0, as the batched entry
    points require.  ``params_list`` holds one parameter set per instance
    (e.g. static-disorder realisations); ``raw_list`` the raw initial MPS of
    each instance.
    """

    def __init__(self, params_list, sites, raw_list, device=0, precision=FP64, kmax=20, tol=0.0,
                 graph=True, stream=None, fused=True, autotune=False, stage3_split=False):
        import torch
        self.torch = torch
        nb = len(params_list)
        self.nb = nb
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.ctx = Context(device, precision, stream=self.stream)
        dev = self.ctx.device
        self.sites = sites
        self.n_e = params_list[0].n_e
        self.kmax, self.tol = kmax, tol
        n = len(sites)
        with torch.cuda.stream(self.stream):
            models = [fmo_model(p, sites) for p in params_list]
            wbond = models[0][1]
            if any(m[1] != wbond for m in models):
                raise TdvpError("instances have different MPO bond dims")
            self.shifts = [m[2] for m in models]
            self.W = [torch.as_tensor(np.stack([m[0][i] for m in models]), dtype=torch.complex128).to(dev)
                      for i in range(n)]
            self.A = [torch.as_tensor(np.stack([r[i] for r in raw_list]), dtype=torch.complex128).to(dev)
                      for i in range(n)]
            bond = [raw_list[0][0].shape[0]] + [a.shape[2] for a in raw_list[0]]
            self.bond, self.wbond = bond, wbond
            et = self.ctx.env_dtype
            self.L = [torch.zeros((nb, bond[b], wbond[b], bond[b]), dtype=et, device=dev) for b in range(n + 1)]
            self.R = [torch.zeros((nb, bond[b], wbond[b], bond[b]), dtype=et, device=dev) for b in range(n + 1)]
            self.obs = torch.zeros((nb, 2 + self.n_e), dtype=torch.float64, device=dev)
        self.stream.synchronize()
        phys = [s[3] for s in sites]
        self._keep = []
        mps_arr = (_Mps * nb)()
        mpo_arr = (_Mpo * nb)()
        env_arr = (_Envs * nb)()
        self.el_sites = [0] * self.n_e
        for i, s in enumerate(sites):
            if s[0] == "el":
                self.el_sites[s[1]] = i
        pp, pb, pw = _i32(phys), _i32(bond), _i32(wbond)
        self._keep += [pp, pb, pw]
        for r in range(nb):
            site = (c_void_p * n)(*[t[r].data_ptr() for t in self.A])
            wsite = (c_void_p * n)(*[t[r].data_ptr() for t in self.W])
            lft = (c_void_p * (n + 1))(*[t[r].data_ptr() for t in self.L])
            rgt = (c_void_p * (n + 1))(*[t[r].data_ptr() for t in self.R])
            self._keep += [site, wsite, lft, rgt]
            mps_arr[r] = _Mps(n, pp, pb, site)
            mpo_arr[r] = _Mpo(n, pp, pw, wsite, float(self.shifts[r]))
            env_arr[r] = _Envs(lft, rgt)
        self.descs = (mps_arr, mpo_arr, env_arr)
        one = workspace_bytes(self.ctx, _Wrap(mps_arr[0]), _Wrap(mpo_arr[0]), kmax)
        self.ctx.reserve(nb * one)
        set_graph(self.ctx, graph)
        set_fused(self.ctx, fused)
        set_stage3_split(self.ctx, stage3_split)
        set_autotune(self.ctx, autotune)
        for r in range(nb):
            _check(lib().tdvp_right_canonicalize(self.ctx.h, ctypes.byref(mps_arr[r])),
                   "tdvp_right_canonicalize")
            _check(lib().tdvp_envs_build(self.ctx.h, ctypes.byref(mps_arr[r]), ctypes.byref(mpo_arr[r]),
                                         ctypes.byref(env_arr[r])), "tdvp_envs_build")

    def step(self, dt_au, nsteps=1):
        ps_step_batched(self.ctx, self.descs, dt_au, nsteps, self.kmax, self.tol)

    def observe(self, out=None):
        out = self.obs if out is None else out
        observe_batched(self.ctx, self.descs, self.el_sites, out)
        return out

    def observe_host(self):
        out = self.observe()
        self.stream.synchronize()
        return out.cpu().numpy().copy()

    def mps_numpy(self, r):
        self.stream.synchronize()
        return [t[r].cpu().numpy() for t in self.A]


class _Wrap:
    """Adapter so workspace_bytes() can take a raw descriptor."""

    def __init__(self, desc):
        self.desc = desc


class DisorderEnsemble:
    """Static-disorder realisations of uneven bond dimension evolved together.

    ``members`` = [(r, params, M_r, raw MPS)] on the chain layout ``sites``;
    realisations that share a bond dimension form one group (one (nb, ...)
    array per site tensor, so the group's chains sit at constant strides).
    With ``grouped=True`` (the default) all groups share one context and
    every step is one tdvp_ps_step_grouped call: each Krylov solve of a
    sweep position is one launch sequence covering every realisation.  With
    ``grouped=False`` each group is a PsEnsemble on a stream of its own
    (groups run concurrently, one launch sequence per group).
    ``observe_host`` returns the observables in realisation order.
    """

    def __init__(self, members, sites, device=0, precision=FP64, kmax=20, tol=0.0, graph=True,
                 fused=True, autotune=False, grouped=True, stage3_split=False):
        import torch
        self.torch = torch
        classes = {}
        for r, p, M, raw in members:
            classes.setdefault(M, []).append((r, p, raw))
        self.nreal = len(members)
        self.grouped = grouped
        self.kmax, self.tol = kmax, tol
        self.classes = []
        if not grouped:
            for M, rs in sorted(classes.items()):
                e = PsEnsemble([p for _, p, _ in rs], sites, [raw for _, _, raw in rs], device, precision,
                               kmax=kmax, tol=tol, graph=graph, fused=fused, autotune=autotune,
                               stage3_split=stage3_split)
                self.classes.append((M, [r for r, _, _ in rs], e))
            self.n_e = self.classes[0][2].n_e
            return
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = Context(device, precision, stream=self.stream)
        dev = self.ctx.device
        n = len(sites)
        self.n_e = members[0][1].n_e
        self.el_sites = [0] * self.n_e
        for i, s_ in enumerate(sites):
            if s_[0] == "el":
                self.el_sites[s_[1]] = i
        phys = [s_[3] for s_ in sites]
        self._keep = []
        self.order = []                   # realisation index of every chain, group-major
        self.counts = []
        groups = sorted(classes.items())
        nb = len(members)
        mps_arr, mpo_arr, env_arr = (_Mps * nb)(), (_Mpo * nb)(), (_Envs * nb)()
        pp = _i32(phys)
        self._keep.append(pp)
        self.tensors = []
        k = 0
        with torch.cuda.stream(self.stream):
            for M, rs in groups:
                models = [fmo_model(p, sites) for _, p, _ in rs]
                wbond = models[0][1]
                if any(m_[1] != wbond for m_ in models):
                    raise TdvpError("realisations have different MPO bond dims")
                W = [torch.as_tensor(np.stack([m_[0][i] for m_ in models]), dtype=torch.complex128).to(dev)
                     for i in range(n)]
                A = [torch.as_tensor(np.stack([raw[i] for _, _, raw in rs]), dtype=torch.complex128).to(dev)
                     for i in range(n)]
                bond = [rs[0][2][0].shape[0]] + [a.shape[2] for a in rs[0][2]]
                et = self.ctx.env_dtype
                L = [torch.zeros((len(rs), bond[b], wbond[b], bond[b]), dtype=et, device=dev) for b in range(n + 1)]
                R = [torch.zeros((len(rs), bond[b], wbond[b], bond[b]), dtype=et, device=dev) for b in range(n + 1)]
                self.tensors.append((M, A, W, L, R))
                pb, pw = _i32(bond), _i32(wbond)
                self._keep += [pb, pw]
                for q, (r, p, raw) in enumerate(rs):
                    site = (c_void_p * n)(*[t[q].data_ptr() for t in A])
                    wsite = (c_void_p * n)(*[t[q].data_ptr() for t in W])
                    lft = (c_void_p * (n + 1))(*[t[q].data_ptr() for t in L])
                    rgt = (c_void_p * (n + 1))(*[t[q].data_ptr() for t in R])
                    self._keep += [site, wsite, lft, rgt]
                    mps_arr[k] = _Mps(n, pp, pb, site)
                    mpo_arr[k] = _Mpo(n, pp, pw, wsite, float(models[q][2]))
                    env_arr[k] = _Envs(lft, rgt)
                    self.order.append(r)
                    k += 1
                self.counts.append(len(rs))
            self.obs = torch.zeros((nb, 2 + self.n_e), dtype=torch.float64, device=dev)
        self.stream.synchronize()
        self.descs = (mps_arr, mpo_arr, env_arr)
        self._counts = _i32(self.counts)
        b = c_size_t(0)
        _check(lib().tdvp_workspace_bytes_grouped(self.ctx.h, len(self.counts), self._counts, mps_arr, mpo_arr,
                                                  kmax, ctypes.byref(b)), "tdvp_workspace_bytes_grouped")
        self.ctx.reserve(b.value)
        set_graph(self.ctx, graph)
        set_fused(self.ctx, fused)
        set_stage3_split(self.ctx, stage3_split)
        set_autotune(self.ctx, autotune)
        for q in range(nb):
            _check(lib().tdvp_right_canonicalize(self.ctx.h, ctypes.byref(mps_arr[q])), "tdvp_right_canonicalize")
            _check(lib().tdvp_envs_build(self.ctx.h, ctypes.byref(mps_arr[q]), ctypes.byref(mpo_arr[q]),
                                         ctypes.byref(env_arr[q])), "tdvp_envs_build")

    def step(self, dt_au, nsteps=1):
        if not self.grouped:
            for _ in range(nsteps):
                for _, _, e in self.classes:
                    e.step(dt_au, 1)
            return
        m, w, e = self.descs
        _check(lib().tdvp_ps_step_grouped(self.ctx.h, len(self.counts), self._counts, m, w, e, float(dt_au),
                                          int(nsteps), int(self.kmax), float(self.tol)), "tdvp_ps_step_grouped")

    def observe_host(self):
        out = np.zeros((self.nreal, 2 + self.n_e))
        if not self.grouped:
            for _, rs, e in self.classes:
                out[rs] = e.observe_host()
            return out
        m, w, e = self.descs
        arr = _i32(self.el_sites)
        _check(lib().tdvp_observe_grouped(self.ctx.h, len(self.counts), self._counts, m, w, e, arr,
                                          len(self.el_sites), _ptr(self.obs)), "tdvp_observe_grouped")
        o = self.obs.cpu().numpy()
        out[self.order] = o
        return out

    def contexts(self):
        """(context, realisations per context) pairs, for kernel timing."""
        if not self.grouped:
            return [(e.ctx, len(rs)) for _, rs, e in self.classes]
        return [(self.ctx, self.nreal)]

    def synchronize(self):
        if not self.grouped:
            for _, _, e in self.classes:
                e.stream.synchronize()
        else:
            self.stream.synchronize()
