"""Thin ctypes binding of libnqs.so (the C ABI in include/nqs.h).

Argument marshalling only: every step of the hot path runs in the library's
gfx950 kernels.  PyTorch supplies device memory and the current HIP stream.
There is no fallback: if the library is missing, importing this module's
functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnqs.so")

NQS_OK, NQS_ERR_ARG, NQS_ERR_DEVICE, NQS_ERR_OOM, NQS_ERR_NONFINITE, NQS_WARN_DEGENERATE, \
    NQS_ERR_NOT_PD, NQS_WARN_NOT_CONVERGED = range(8)
PRECISION = {"fp64": 0, "fp32": 1, "bf16x2": 2}
IRREP = {"A1": 0, "A2": 1, "B1": 2, "B2": 3}
OP = {"logpsi": 0, "eloc": 1, "moments": 2, "grad": 3, "sr": 4, "sample": 5, "sq": 6, "vmc": 7, "cg": 8,
      "moments2": 9, "eloc_grad": 10}

EXPORTS = ["nqs_create", "nqs_destroy", "nqs_num_params", "nqs_workspace_bytes", "nqs_set_params",
           "nqs_logpsi", "nqs_eloc", "nqs_eloc_noalloc", "nqs_lanczos_moments", "nqs_lanczos_moments_p2", "nqs_grad", "nqs_eloc_grad", "nqs_sr_solve",
           "nqs_chain_init", "nqs_sample", "nqs_enumerate_sz0", "nqs_set_factor_form",
           "nqs_structure_factor", "nqs_get_params", "nqs_vmc_step", "nqs_sr_solve_cg",
           "nqs_profile_enable", "nqs_profile_read", "nqs_status_str", "nqs_last_error"]
KERNELS = {"theta": 0, "lse": 1, "eloc_bonds": 2, "eloc_finish": 3, "twohop": 4,
           "twohop_finish": 5, "moments": 6, "grad": 7, "sample": 8, "sr": 9, "gram": 10,
           "cholesky": 11, "sq": 12, "cg": 13, "hop3": 14}


class ModelDesc(C.Structure):
    _fields_ = [("L", C.c_int32), ("J1", C.c_double), ("J2", C.c_double), ("kx", C.c_int32),
                ("ky", C.c_int32), ("irrep", C.c_int32), ("n_rbm", C.c_int32),
                ("n_hidden", C.c_int32), ("use_bias", C.c_int32), ("precision", C.c_int32)]


class Moments(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_double) for k in (
        "h1", "h1_im", "h2", "h2_alt", "h3", "c2", "c3", "v", "r", "alpha", "e_p1", "h1_err")] + [
        ("degenerate", C.c_int32)]


class Moments2(C.Structure):
    _fields_ = [("p1", Moments)] + [(k, C.c_double) for k in (
        "h4", "h5", "mu4", "mu5", "e_p2", "beta1", "beta2")] + [("degenerate", C.c_int32)]


class VmcStats(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_double) for k in (
        "energy", "energy_im", "variance", "error", "dtheta_norm")] + [
        ("solver_iters", C.c_int32), ("solver_resid", C.c_double)]


class NQSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnqs.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2206_14307_amd.build.build()")
    lib = C.CDLL(path)
    vp, i64, i32, u64, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
    sig = {
        "nqs_create": ([C.POINTER(ModelDesc), C.POINTER(vp)], C.c_int),
        "nqs_destroy": ([vp], None),
        "nqs_num_params": ([vp], i64),
        "nqs_workspace_bytes": ([vp, C.c_int, i64], C.c_size_t),
        "nqs_set_params": ([vp, vp, vp], C.c_int),
        "nqs_logpsi": ([vp, vp, i64, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_eloc": ([vp, vp, i64, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_eloc_noalloc": ([vp, vp, i64, vp, vp, vp], C.c_int),
        "nqs_lanczos_moments": ([vp, vp, i64, C.c_int, vp, C.POINTER(Moments), vp, C.c_size_t, vp],
                                C.c_int),
        "nqs_lanczos_moments_p2": ([vp, vp, i64, C.c_int, vp, C.POINTER(Moments2), vp, C.c_size_t,
                                    vp], C.c_int),
        "nqs_grad": ([vp, vp, i64, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_eloc_grad": ([vp, vp, i64, vp, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_sr_solve": ([vp, vp, vp, i64, dbl, dbl, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_chain_init": ([vp, vp, i64, u64, vp, vp], C.c_int),
        "nqs_sample": ([vp, i64, i64, i32, i32, u64, vp, vp, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_enumerate_sz0": ([vp, vp, i64, C.POINTER(i64), vp], C.c_int),
        "nqs_set_factor_form": ([vp, C.c_int], C.c_int),
        "nqs_structure_factor": ([vp, vp, i64, vp, vp, vp, C.c_size_t, vp], C.c_int),
        "nqs_get_params": ([vp, vp, vp], C.c_int),
        "nqs_sr_solve_cg": ([vp, vp, vp, i64, dbl, dbl, dbl, C.c_int, vp, C.POINTER(C.c_int),
                             C.POINTER(dbl), vp, C.c_size_t, vp], C.c_int),
        "nqs_vmc_step": ([vp, vp, i64, dbl, dbl, C.c_int, C.c_int, C.POINTER(VmcStats), vp,
                          C.c_size_t, vp], C.c_int),
        "nqs_profile_enable": ([vp, C.c_int], C.c_int),
        "nqs_profile_read": ([vp, C.c_int, C.POINTER(dbl), C.POINTER(i64), C.c_int], C.c_int),
        "nqs_status_str": ([C.c_int], C.c_char_p),
        "nqs_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class NQS:
    """One model context (lattice tables + parameters) on the current device."""

    def __init__(self, L, J1=1.0, J2=0.5, kx=0, ky=0, irrep="A1", n_rbm=1, n_hidden=16,
                 use_bias=True, precision="fp32", device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        self.L, self.N = L, L * L
        self.G = 8 * self.N
        self.n_rbm, self.n_hidden = n_rbm, n_hidden
        self.precision = precision
        irrep_id = IRREP[irrep] if isinstance(irrep, str) else int(irrep)
        self.desc = ModelDesc(L, J1, J2, kx, ky, irrep_id, n_rbm, n_hidden, int(bool(use_bias)),
                              PRECISION[precision])
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.nqs_create(C.byref(self.desc), C.byref(self._ctx))
        if st != NQS_OK:
            raise NQSError(st, f"nqs_create failed: {self.lib.nqs_status_str(st).decode()}")
        self.P = int(self.lib.nqs_num_params(self._ctx))
        self._ws = None
        self.last_status = NQS_OK

    @classmethod
    def from_workload(cls, w, device="cuda"):
        return cls(w.L, w.J1, w.J2, w.kx, w.ky, w.irrep, w.n_rbm, w.n_hidden, w.use_bias,
                   w.precision, device)

    def close(self):
        if self._ctx:
            self.lib.nqs_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _check(self, st, what):
        """Raise on an error status; warnings (degenerate Lanczos step, CG
        stopped above its tolerance) are kept in ``last_status``."""
        self.last_status = st
        if st not in (NQS_OK, NQS_WARN_DEGENERATE, NQS_WARN_NOT_CONVERGED):
            msg = self.lib.nqs_last_error(self._ctx).decode()
            raise NQSError(st, f"{what}: {self.lib.nqs_status_str(st).decode()}: {msg}")
        return st

    def workspace(self, op, S):
        need = int(self.lib.nqs_workspace_bytes(self._ctx, OP[op], int(S)))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def _spins(self, spins):
        spins = torch.as_tensor(spins)
        if spins.dtype != torch.int8:
            spins = spins.to(torch.int8)
        spins = spins.to(self.device).contiguous()
        if spins.dim() != 2 or spins.shape[1] != self.N:
            raise ValueError(f"spins must be [S, {self.N}] int8")
        return spins

    @property
    def o_dtype(self):
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    # ----------------------------------------------------------------- calls
    def set_params(self, params):
        p = torch.as_tensor(params).to(torch.complex128).reshape(-1).to(self.device).contiguous()
        if p.numel() != self.P:
            raise ValueError(f"expected {self.P} parameters, got {p.numel()}")
        self._check(self.lib.nqs_set_params(self._ctx, _ptr(torch.view_as_real(p)), _stream()),
                    "nqs_set_params")

    def get_params(self):
        """The context's current parameters, complex128 [P] (nqs_set_params layout)."""
        out = torch.empty(self.P, dtype=torch.complex128, device=self.device)
        self._check(self.lib.nqs_get_params(self._ctx, _ptr(torch.view_as_real(out)), _stream()),
                    "nqs_get_params")
        return out

    def vmc_step(self, spins, lam=1e-6, dtau=0.01, real_params=False, solver="cholesky"):
        """One SR training step on the configurations (nqs_vmc_step): returns the
        energy statistics of the parameters before the update.  solver:
        "cholesky" (sample space) or "cg" (parameter space)."""
        code = {"cholesky": 0, "cg": 1}[solver]
        sp = self._spins(spins)
        S = sp.shape[0]
        ws = self.workspace("vmc", S)
        st = VmcStats()
        self._check(self.lib.nqs_vmc_step(self._ctx, _ptr(sp), S, float(lam), float(dtau),
                                          int(bool(real_params)), code, C.byref(st), _ptr(ws),
                                          ws.numel(), _stream()), "nqs_vmc_step")
        return {k: getattr(st, k) for k, _ in VmcStats._fields_}

    def set_factor_form(self, direct_only):
        self._check(self.lib.nqs_set_factor_form(self._ctx, int(bool(direct_only))),
                    "nqs_set_factor_form")

    def sector_size(self):
        n = C.c_int64(0)
        self._check(self.lib.nqs_enumerate_sz0(self._ctx, None, 0, C.byref(n), _stream()),
                    "nqs_enumerate_sz0")
        return n.value

    def enumerate_sz0(self):
        """All Sz = 0 configurations [C(N, N/2)][N] int8 in colex order."""
        D = self.sector_size()
        out = torch.empty((D, self.N), dtype=torch.int8, device=self.device)
        n = C.c_int64(0)
        self._check(self.lib.nqs_enumerate_sz0(self._ctx, _ptr(out), D, C.byref(n), _stream()),
                    "nqs_enumerate_sz0")
        return out

    def structure_factor(self, spins, weights=None):
        """S(q) for every momentum q = 2 pi (kx, ky) / L (index kx + L ky), float64 [N]:
        the mean over the configurations, weighted by `weights` (FP64 [S], e.g.
        |psi|^2) when given.  The paper's tables show N S(q)."""
        sp = self._spins(spins)
        S = sp.shape[0]
        w = None
        if weights is not None:
            w = torch.as_tensor(weights, dtype=torch.float64).to(self.device).contiguous()
            if w.shape != (S,):
                raise ValueError(f"weights must be float64 [{S}]")
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        ws = self.workspace("sq", S)
        self._check(self.lib.nqs_structure_factor(self._ctx, _ptr(sp), S, _ptr(w), _ptr(out),
                                                  _ptr(ws), ws.numel(), _stream()),
                    "nqs_structure_factor")
        return out

    def logpsi(self, spins):
        sp = self._spins(spins)
        S = sp.shape[0]
        out = torch.empty(S, dtype=torch.complex128, device=self.device)
        ws = self.workspace("logpsi", S)
        self._check(self.lib.nqs_logpsi(self._ctx, _ptr(sp), S, _ptr(out), _ptr(ws), ws.numel(),
                                        _stream()), "nqs_logpsi")
        return out

    def eloc(self, spins, want_logpsi=True):
        sp = self._spins(spins)
        S = sp.shape[0]
        el = torch.empty(S, dtype=torch.complex128, device=self.device)
        lp = torch.empty(S, dtype=torch.complex128, device=self.device) if want_logpsi else None
        ws = self.workspace("eloc", S)
        self._check(self.lib.nqs_eloc(self._ctx, _ptr(sp), S, _ptr(lp), _ptr(el), _ptr(ws),
                                      ws.numel(), _stream()), "nqs_eloc")
        return (lp, el) if want_logpsi else el

    def lanczos_moments(self, spins, exact=False, want_e1e2=True):
        sp = self._spins(spins)
        S = sp.shape[0]
        e12 = torch.empty((S, 2), dtype=torch.complex128, device=self.device) if want_e1e2 else None
        ws = self.workspace("moments", S)
        m = Moments()
        st = self._check(self.lib.nqs_lanczos_moments(self._ctx, _ptr(sp), S, int(bool(exact)),
                                                      _ptr(e12), C.byref(m), _ptr(ws), ws.numel(),
                                                      _stream()), "nqs_lanczos_moments")
        res = {k: getattr(m, k) for k, _ in Moments._fields_}
        res["degenerate"] = bool(res["degenerate"])
        res["status"] = st
        return res, e12

    def lanczos_moments_p2(self, spins, exact=False, want_e123=True):
        """Moments to fifth order and the p = 2 Lanczos energy; returns
        (dict, e123) with e123 complex128 [S][3] = (e1, e2, e3) or None.  The
        dict holds the p = 1 fields and h4 h5 mu4 mu5 e_p2 beta1 beta2;
        degenerate / degenerate1 are the p = 2 / p = 1 flags."""
        sp = self._spins(spins)
        S = sp.shape[0]
        e123 = torch.empty((S, 3), dtype=torch.complex128, device=self.device) if want_e123 else None
        ws = self.workspace("moments2", S)
        m = Moments2()
        st = self._check(self.lib.nqs_lanczos_moments_p2(self._ctx, _ptr(sp), S, int(bool(exact)),
                                                         _ptr(e123), C.byref(m), _ptr(ws),
                                                         ws.numel(), _stream()),
                         "nqs_lanczos_moments_p2")
        res = {k: getattr(m.p1, k) for k, _ in Moments._fields_}
        res["degenerate1"] = bool(res.pop("degenerate"))
        res.update({k: getattr(m, k) for k, _ in Moments2._fields_[1:]})
        res["degenerate"] = bool(res["degenerate"])
        res["status"] = st
        return res, e123

    def grad(self, spins, want_logpsi=False):
        sp = self._spins(spins)
        S = sp.shape[0]
        O = torch.empty((S, self.P), dtype=self.o_dtype, device=self.device)
        lp = torch.empty(S, dtype=torch.complex128, device=self.device) if want_logpsi else None
        ws = self.workspace("grad", S)
        self._check(self.lib.nqs_grad(self._ctx, _ptr(sp), S, _ptr(O), _ptr(lp), _ptr(ws),
                                      ws.numel(), _stream()), "nqs_grad")
        return (O, lp) if want_logpsi else O

    def eloc_grad(self, spins, want_logpsi=True):
        """(log psi, E_loc, O) of the same configurations in one call
        (nqs_eloc_grad); (E_loc, O) without log psi."""
        sp = self._spins(spins)
        S = sp.shape[0]
        el = torch.empty(S, dtype=torch.complex128, device=self.device)
        lp = torch.empty(S, dtype=torch.complex128, device=self.device) if want_logpsi else None
        O = torch.empty((S, self.P), dtype=self.o_dtype, device=self.device)
        ws = self.workspace("eloc_grad", S)
        self._check(self.lib.nqs_eloc_grad(self._ctx, _ptr(sp), S, _ptr(lp), _ptr(el), _ptr(O),
                                           _ptr(ws), ws.numel(), _stream()), "nqs_eloc_grad")
        return (lp, el, O) if want_logpsi else (el, O)

    def sr_solve(self, O, eloc, lam=1e-6, dtau=0.01):
        S = O.shape[0]
        O = O.to(self.o_dtype).contiguous()
        el = eloc.to(torch.complex128).contiguous()
        out = torch.empty(self.P, dtype=torch.complex128, device=self.device)
        ws = self.workspace("sr", S)
        self._check(self.lib.nqs_sr_solve(self._ctx, _ptr(O), _ptr(el), S, float(lam), float(dtau),
                                          _ptr(out), _ptr(ws), ws.numel(), _stream()),
                    "nqs_sr_solve")
        return out

    def sr_solve_cg(self, O, eloc, lam=1e-6, dtau=0.01, tol=1e-10, max_iter=1000):
        """Eq. (12) by matrix-free conjugate gradients in parameter space:
        returns (dtheta complex128 [P], iterations, relative residual)."""
        S = O.shape[0]
        O = O.to(self.o_dtype).contiguous()
        el = eloc.to(torch.complex128).contiguous()
        out = torch.empty(self.P, dtype=torch.complex128, device=self.device)
        ws = self.workspace("cg", S)
        it, res = C.c_int(0), C.c_double(0.0)
        self._check(self.lib.nqs_sr_solve_cg(self._ctx, _ptr(O), _ptr(el), S, float(lam),
                                             float(dtau), float(tol), int(max_iter), _ptr(out),
                                             C.byref(it), C.byref(res), _ptr(ws), ws.numel(),
                                             _stream()), "nqs_sr_solve_cg")
        return out, it.value, res.value

    def chain_init(self, spins, first_chain_id=0):
        sp = self._spins(spins)
        n = sp.shape[0]
        state = torch.empty((n, 4), dtype=torch.int64, device=self.device)
        self._check(self.lib.nqs_chain_init(self._ctx, _ptr(sp), n, int(first_chain_id),
                                            _ptr(state), _stream()), "nqs_chain_init")
        return state

    def sample(self, state, n_per_chain, n_skip=0, n_burn=0, seed=0):
        n = state.shape[0]
        spins = torch.empty((n * n_per_chain, self.N), dtype=torch.int8, device=self.device)
        acc = torch.empty(n, dtype=torch.float32, device=self.device)
        nskip = torch.zeros(1, dtype=torch.int32, device=self.device)
        ws = self.workspace("sample", n)
        self._check(self.lib.nqs_sample(self._ctx, n, int(n_per_chain), int(n_skip), int(n_burn),
                                        int(seed), _ptr(state), _ptr(spins), _ptr(acc),
                                        _ptr(nskip), _ptr(ws), ws.numel(), _stream()),
                    "nqs_sample")
        return spins, acc, nskip


    # ------------------------------------------------------------ profiling
    def profile(self, on=True):
        self._check(self.lib.nqs_profile_enable(self._ctx, int(bool(on))), "nqs_profile_enable")

    def profile_read(self, kernel, reset=True):
        """(total ms, launches) of one kernel since the last reset."""
        ms, n = C.c_double(), C.c_int64()
        self._check(self.lib.nqs_profile_read(self._ctx, KERNELS[kernel], C.byref(ms), C.byref(n),
                                              int(bool(reset))), "nqs_profile_read")
        return ms.value, n.value


class LogPsi(torch.autograd.Function):
    """log psi(sigma; theta) with the hand-written backward O_k (nqs_grad).

    ``LogPsi.apply(params, spins, model)`` evaluates log psi at ``params``
    (complex [P], or real [P] for a real RBM) and leaves the context's own
    parameters as they were.  The forward forms O_k (nqs_grad) only when a
    gradient with respect to params is wanted, else it calls nqs_logpsi.

    PyTorch's complex convention: for the holomorphic map theta -> log psi,
    the vector-Jacobian product is grad_theta_k = sum_s grad_out[s] conj(O[s, k]);
    for real parameters it is the real part of that sum."""

    @staticmethod
    def forward(ctx, params, spins, model):
        prev = model.get_params()
        p = params.detach().reshape(-1).to(device=prev.device, dtype=torch.complex128)
        changed = not torch.equal(prev, p)
        if changed:
            model.set_params(p)
        try:
            if ctx.needs_input_grad[0]:
                O, lp = model.grad(spins, want_logpsi=True)
                ctx.save_for_backward(O)
            else:
                lp = model.logpsi(spins)
        finally:
            if changed:
                model.set_params(prev)
        ctx.real_params = not params.is_complex()
        ctx.shape, ctx.dtype = params.shape, params.dtype
        return lp

    @staticmethod
    def backward(ctx, grad_out):
        (O,) = ctx.saved_tensors
        g = grad_out.to(torch.complex128)
        gp = (g[:, None] * O.to(torch.complex128).conj()).sum(dim=0)
        if ctx.real_params:
            gp = gp.real
        return gp.reshape(ctx.shape).to(ctx.dtype), None, None
