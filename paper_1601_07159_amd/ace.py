"""Python binding of libace over PyTorch device tensors.

Argument marshalling only: every step runs in the HIP kernels of libace.so.
PyTorch supplies device memory and the current HIP stream.  There is no CPU
path; calling these functions without the built library or on CPU tensors
raises.

Orbital blocks are complex tensors of shape (N, n0, n1, n2) (or (N, N_g)) whose
last dimensions are contiguous; the stride of dim 0 is the C ABI's ``ld``.
complex128 goes with FP64, complex64 with FP32 and MIXED; real orbitals
(precisions "real64" / "real32") are float64 / float32 tensors of the same
shapes.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import ACE_FP32, ACE_FP64, ACE_MIXED, ACE_REAL32, ACE_REAL64  # noqa: F401

PREC = {"fp64": ACE_FP64, "fp32": ACE_FP32, "mixed": ACE_MIXED, "real64": ACE_REAL64,
        "real32": ACE_REAL32}
_TUNE_KEYS = {"pair_budget": _lib.ACE_TUNE_PAIR_BUDGET, "jblock": _lib.ACE_TUNE_JBLOCK,
              "symmetry": _lib.ACE_TUNE_SYMMETRY, "fft_shape": _lib.ACE_TUNE_FFT_SHAPE,
              "accum_shape": _lib.ACE_TUNE_ACCUM_SHAPE, "branches": _lib.ACE_TUNE_BRANCHES,
              "batch_form": _lib.ACE_TUNE_BATCH_FORM}


class AceError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


@dataclass(frozen=True)
class Grid:
    """Cubic grid n^3 in an orthorhombic cell L (bohr); kind 'coulomb' or 'erfc'."""
    n: int
    L: tuple
    kind: str = "coulomb"
    mu: float = 0.0
    g0: float = 0.0

    @staticmethod
    def cubic(n: int, L: float, kind: str = "coulomb", mu: float = 0.0, g0: float = 0.0):
        return Grid(int(n), (float(L),) * 3, kind, float(mu), float(g0))

    @property
    def ng(self) -> int:
        return self.n ** 3

    @property
    def omega(self) -> float:
        return self.L[0] * self.L[1] * self.L[2]

    @property
    def dV(self) -> float:
        return self.omega / self.ng

    def as_c(self) -> _lib.AceGrid:
        g = _lib.AceGrid()
        for a in range(3):
            g.n[a] = self.n
            g.L[a] = float(self.L[a])
        g.kind = {"coulomb": _lib.ACE_COULOMB, "erfc": _lib.ACE_ERFC}[self.kind]
        g.mu = float(self.mu)
        g.g0 = float(self.g0)
        return g


def _prec(p) -> int:
    if isinstance(p, str):
        return PREC[p.lower()]
    return int(p)


def _dtype_for(prec: int):
    return {ACE_FP64: torch.complex128, ACE_REAL64: torch.float64,
            ACE_REAL32: torch.float32}.get(prec, torch.complex64)


def _block(t: torch.Tensor, prec: int, ng: int, what: str):
    """(pointer, count, ld) of an orbital block; validates device/dtype/layout."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a GPU tensor")
    if t.dtype != _dtype_for(prec):
        raise TypeError(f"{what}: dtype {t.dtype} does not match precision "
                        f"(expected {_dtype_for(prec)})")
    if t.dim() < 2:
        raise ValueError(f"{what}: expected (N, n0, n1, n2) or (N, N_g)")
    count = t.shape[0]
    inner = 1
    for s in t.shape[1:]:
        inner *= s
    if inner != ng:
        raise ValueError(f"{what}: {inner} grid values per orbital, grid has {ng}")
    flat = t.reshape(count, ng) if t.is_contiguous() else None
    if flat is None:
        # require each orbital contiguous
        exp = 1
        for d in range(t.dim() - 1, 0, -1):
            if t.shape[d] != 1 and t.stride(d) != exp:
                raise ValueError(f"{what}: each orbital must be contiguous")
            exp *= t.shape[d]
    return ctypes.c_void_p(t.data_ptr()), int(count), int(t.stride(0))


class Context:
    """An ace_ctx bound to one device; calls run on torch's current stream."""

    def __init__(self, device=None, tune_cache=None):
        self._lib = _lib.load()
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        self.device = dev
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = self._lib.ace_create(ctypes.byref(h), ctypes.c_void_p(
                torch.cuda.current_stream(dev).cuda_stream),
                tune_cache.encode() if tune_cache else None)
        if st != 0:
            raise AceError(st, "ace_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plumbing -------------------------------------------------------------
    def _bind_stream(self):
        self._lib.ace_set_stream(self._h, ctypes.c_void_p(
            torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, st: int):
        if st != 0:
            msg = self._lib.ace_last_error(self._h).decode()
            name = self._lib.ace_status_string(st).decode()
            raise AceError(st, f"{name}: {msg}")

    # -- entry points ---------------------------------------------------------
    def reserve(self, grid: Grid, prec, max_nocc: int, max_nband: int, max_nx: int = 0):
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_reserve(self._h, ctypes.byref(g), _prec(prec), max_nocc,
                                          max_nband, max_nx))

    def set_pair_budget(self, nbytes: int):
        self._check(self._lib.ace_set_pair_budget(self._h, int(nbytes)))

    def set_tuning(self, key: str, value: int):
        self._check(self._lib.ace_set_tuning(self._h, _TUNE_KEYS[key], int(value)))

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_long()
        self._check(self._lib.ace_get_tuning(self._h, _TUNE_KEYS[key], ctypes.byref(v)))
        return v.value

    def build_W(self, phi, psi, grid: Grid, prec, scale: float = 1.0, out=None):
        """W = scale * V_X[phi] psi (pair Poisson solves)."""
        p = _prec(prec)
        a, na, lda = _block(phi, p, grid.ng, "phi")
        b, nb, ldb = _block(psi, p, grid.ng, "psi")
        if out is None:
            out = torch.empty_like(psi, memory_format=torch.contiguous_format)
        w, nw, ldw = _block(out, p, grid.ng, "W")
        if nw != nb:
            raise ValueError("W must hold n_band orbitals")
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_build_W(self._h, ctypes.byref(g), p, a, na, lda, b, nb, ldb, w,
                                          ldw, float(scale)))
        return out

    def compress(self, psi, W, grid: Grid, prec, want_L: bool = False, info=None, out=None):
        """xi = W L^{-H} with -<psi, W> = L L^H.  Returns xi (and L when want_L)."""
        p = _prec(prec)
        a, na, lda = _block(psi, p, grid.ng, "psi")
        w, nw, ldw = _block(W, p, grid.ng, "W")
        if nw != na:
            raise ValueError("psi and W must hold the same number of orbitals")
        if out is None:
            out = torch.empty_like(W, memory_format=torch.contiguous_format)
        x, nx, ldx = _block(out, p, grid.ng, "xi")
        L = torch.empty((na, na), dtype=torch.complex128, device=W.device) if want_L else None
        Lp = ctypes.c_void_p(L.data_ptr()) if L is not None else None
        ip = None
        if info is not None:
            if info.dtype != torch.int32 or not info.is_cuda:
                raise TypeError("info must be a CUDA int32 tensor")
            ip = ctypes.c_void_p(info.data_ptr())
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_compress(self._h, ctypes.byref(g), p, a, lda, w, ldw, na, x,
                                           ldx, Lp, ip))
        if want_L:
            # column-major n x n  ->  row-major view of L
            return out, L.t().contiguous()
        return out

    def apply(self, xi, X, grid: Grid, prec, out=None):
        """Y = -xi (dV xi^H X)."""
        p = _prec(prec)
        a, na, lda = _block(xi, p, grid.ng, "xi")
        b, nb, ldb = _block(X, p, grid.ng, "X")
        if out is None:
            out = torch.empty_like(X, memory_format=torch.contiguous_format)
        y, ny, ldy = _block(out, p, grid.ng, "Y")
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_apply(self._h, ctypes.byref(g), p, a, na, lda, b, nb, ldb, y,
                                        ldy))
        return out

    def exchange_energy(self, phi, grid: Grid, prec, xi=None, out=None):
        """E_X as a 0-dim float64 device tensor (from xi when given, else directly)."""
        p = _prec(prec)
        a, na, lda = _block(phi, p, grid.ng, "phi")
        if xi is not None:
            b, nb, ldb = _block(xi, p, grid.ng, "xi")
        else:
            b, nb, ldb = None, 0, 0
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=phi.device)
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_exchange_energy(self._h, ctypes.byref(g), p, a, na, lda, b, nb,
                                                  ldb, ctypes.c_void_p(out.data_ptr())))
        return out

    def exchange_energy_grad(self, phi, grid: Grid, prec, gbar=None, out=None):
        """G = 2 gbar dV V_X[phi] phi (PyTorch's gradient of E_X for complex phi)."""
        p = _prec(prec)
        a, na, lda = _block(phi, p, grid.ng, "phi")
        if out is None:
            out = torch.empty_like(phi, memory_format=torch.contiguous_format)
        o, no, ldo = _block(out, p, grid.ng, "G")
        gp = None
        if gbar is not None:
            if gbar.dtype != torch.float64 or not gbar.is_cuda or gbar.numel() != 1:
                raise TypeError("gbar must be a one-element CUDA float64 tensor")
            gp = ctypes.c_void_p(gbar.data_ptr())
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_exchange_energy_grad(self._h, ctypes.byref(g), p, a, na, lda,
                                                       gp, o, ldo))
        return out

    def orthonormalize(self, X, grid: Grid, prec, info=None, out=None):
        p = _prec(prec)
        a, na, lda = _block(X, p, grid.ng, "X")
        if out is None:
            out = torch.empty_like(X, memory_format=torch.contiguous_format)
        q, nq, ldq = _block(out, p, grid.ng, "Q")
        ip = ctypes.c_void_p(info.data_ptr()) if info is not None else None
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_orthonormalize(self._h, ctypes.byref(g), p, a, na, lda, q, ldq,
                                                 ip))
        return out

    def apply_h(self, X, grid: Grid, prec, vloc=None, xi=None, phi=None, scale_x: float = 1.0,
                out=None):
        """Y = (-1/2 Laplacian + V_loc) X + V_ex X with V_ex = V_ACE (xi given),
        scale_x V_X[phi] (phi given) or none (ace_apply_h)."""
        p = _prec(prec)
        x, nx, ldx = _block(X, p, grid.ng, "X")
        if out is None:
            out = torch.empty_like(X, memory_format=torch.contiguous_format)
        y, ny, ldy = _block(out, p, grid.ng, "Y")
        vp = None
        if vloc is not None:
            want = torch.float64 if p == ACE_FP64 else torch.float32
            if vloc.dtype != want or not vloc.is_cuda or vloc.numel() != grid.ng or \
                    not vloc.is_contiguous():
                raise TypeError(f"vloc must be a contiguous CUDA {want} tensor of N_g values")
            vp = ctypes.c_void_p(vloc.data_ptr())
        xp, nxi, ldxi = _block(xi, p, grid.ng, "xi") if xi is not None else (None, 0, 0)
        pp, nph, ldph = _block(phi, p, grid.ng, "phi") if phi is not None else (None, 0, 0)
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_apply_h(self._h, ctypes.byref(g), p, vp, xp, nxi, ldxi, pp, nph,
                                          ldph, float(scale_x), x, nx, ldx, y, ldy))
        return out

    def combine(self, grid: Grid, prec, a, A, b=0.0, B=None, c=0.0, C=None, out=None):
        """D = a A + b B + c C on orbital blocks (ace_combine)."""
        p = _prec(prec)
        ap, n, lda = _block(A, p, grid.ng, "A")
        bp, _, ldb = _block(B, p, grid.ng, "B") if B is not None else (None, 0, 0)
        cp, _, ldc = _block(C, p, grid.ng, "C") if C is not None else (None, 0, 0)
        if out is None:
            out = torch.empty_like(A, memory_format=torch.contiguous_format)
        dp, _, ldd = _block(out, p, grid.ng, "D")
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_combine(self._h, ctypes.byref(g), p, n, float(a), ap, lda,
                                          float(b), bp, ldb, float(c), cp, ldc, dp, ldd))
        return out

    def rayleigh_ritz(self, X, HX, grid: Grid, prec, out_X=None, out_HX=None, evals=None):
        """Ritz pairs of H on span(X) (X orthonormal, HX = H X): returns
        (X Q, HX Q, eigenvalues ascending as a float64 device tensor)."""
        p = _prec(prec)
        x, n, ldx = _block(X, p, grid.ng, "X")
        h, nh, ldh = _block(HX, p, grid.ng, "HX")
        if nh != n:
            raise ValueError("X and HX must hold the same number of orbitals")
        if out_X is None:
            out_X = torch.empty_like(X, memory_format=torch.contiguous_format)
        if out_HX is None:
            out_HX = torch.empty_like(X, memory_format=torch.contiguous_format)
        ox, _, ldo = _block(out_X, p, grid.ng, "Xout")
        oh, _, ldo2 = _block(out_HX, p, grid.ng, "HXout")
        if ldo2 != ldo:
            raise ValueError("out_X and out_HX need the same leading dimension")
        if evals is None:
            evals = torch.empty(n, dtype=torch.float64, device=X.device)
        g = grid.as_c()
        self._bind_stream()
        self._check(self._lib.ace_rayleigh_ritz(self._h, ctypes.byref(g), p, x, ldx, h, ldh, n, ox,
                                                oh, ldo, ctypes.c_void_p(evals.data_ptr())))
        return out_X, out_HX, evals

    def build_batched(self, instances, prec, n_branches: int = None):
        """Build W (and xi when an instance has one) for many independent systems
        (ace_build_W_batched).

        ``instances``: list of dicts with keys grid (Grid), phi, psi, W, and
        optionally xi, info (CUDA int32, required with xi), scale and prec
        (default: ``prec``).  n_branches (optional) sets the tuning knob of
        the branch streams.  The first call captures a HIP graph; identical
        later calls replay it."""
        if n_branches is not None:
            self.set_tuning("branches", int(n_branches))
        arr = (_lib.AceInstance * len(instances))()
        self._keep = []
        for k, d in enumerate(instances):
            g = d["grid"]
            p = _prec(d.get("prec", prec))
            a, na, lda = _block(d["phi"], p, g.ng, "phi")
            b, nb, ldb = _block(d["psi"], p, g.ng, "psi")
            w, nw, ldw = _block(d["W"], p, g.ng, "W")
            if nw != nb:
                raise ValueError("W must hold n_band orbitals")
            e = arr[k]
            e.grid = g.as_c()
            e.prec = p
            e.phi, e.n_occ, e.ld_phi = a, na, lda
            e.psi, e.n_band, e.ld_psi = b, nb, ldb
            e.W, e.ld_W = w, ldw
            xi = d.get("xi")
            if xi is not None:
                x, nx, ldx = _block(xi, p, g.ng, "xi")
                info = d["info"]
                if info.dtype != torch.int32 or not info.is_cuda:
                    raise TypeError("info must be a CUDA int32 tensor")
                e.xi, e.ld_xi = x, ldx
                e.info_dev = ctypes.c_void_p(info.data_ptr())
            else:
                e.xi, e.ld_xi, e.info_dev = None, 0, None
            e.scale = float(d.get("scale", 1.0))
        self._bind_stream()
        self._check(self._lib.ace_build_W_batched(self._h, len(instances), arr))

    def autotune(self, grid: Grid, prec, n_occ: int, n_band: int, cache_path=None) -> dict:
        """Time the build over pair budgets, band blocks and FFT line shapes; keep
        the fastest for this grid size (ace_autotune)."""
        g = grid.as_c()
        bud, jb, sh, ac = ctypes.c_long(), ctypes.c_long(), ctypes.c_int(), ctypes.c_int()
        ms = ctypes.c_double()
        self._bind_stream()
        self._check(self._lib.ace_autotune(
            self._h, ctypes.byref(g), _prec(prec), int(n_occ), int(n_band),
            cache_path.encode() if cache_path else None, ctypes.byref(bud), ctypes.byref(jb),
            ctypes.byref(sh), ctypes.byref(ac), ctypes.byref(ms)))
        return {"pair_budget": bud.value, "jblock": jb.value, "fft_shape": sh.value,
                "accum_shape": ac.value, "ms": ms.value}

    def tune_load(self, cache_path: str):
        self._check(self._lib.ace_tune_load(self._h, cache_path.encode()))

    # -- profiling ------------------------------------------------------------
    def profile(self, on: bool = True):
        self._check(self._lib.ace_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        self._check(self._lib.ace_profile_reset(self._h))

    def profile_report(self) -> dict:
        out = {}
        for k in range(self._lib.ace_profile_count(self._h)):
            name = ctypes.c_char_p()
            launches = ctypes.c_long()
            ms = ctypes.c_double()
            self._check(self._lib.ace_profile_get(self._h, k, ctypes.byref(name),
                                                  ctypes.byref(launches), ctypes.byref(ms)))
            out[name.value.decode()] = {"launches": launches.value, "ms": ms.value}
        return out


_default = {}


def context(device=None) -> Context:
    idx = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    if idx not in _default:
        _default[idx] = Context(idx)
    return _default[idx]


def supported_n():
    lib = _lib.load()
    buf = (ctypes.c_int * 64)()
    k = lib.ace_supported_n(buf, 64)
    return [buf[i] for i in range(k)]


def build_W(phi, psi, grid, prec, scale=1.0, out=None):
    return context(phi.device).build_W(phi, psi, grid, prec, scale, out)


def compress(psi, W, grid, prec, want_L=False, info=None, out=None):
    return context(W.device).compress(psi, W, grid, prec, want_L, info, out)


def apply(xi, X, grid, prec, out=None):
    return context(X.device).apply(xi, X, grid, prec, out)


def exchange_energy(phi, grid, prec, xi=None, out=None):
    return context(phi.device).exchange_energy(phi, grid, prec, xi, out)


def orthonormalize(X, grid, prec, info=None, out=None):
    return context(X.device).orthonormalize(X, grid, prec, info, out)


def exchange_energy_grad(phi, grid, prec, gbar=None, out=None):
    return context(phi.device).exchange_energy_grad(phi, grid, prec, gbar, out)


class ExchangeEnergy(torch.autograd.Function):
    """E_X(phi) = 1/2 sum_i <phi_i, V_X[phi] phi_i> with a hand-written backward.

    forward: Parseval sum over the pair spectra i <= j (forward FFTs only);
    backward: the orbital gradient 2 gbar dV V_X[phi] phi, recomputing the
    pair FFTs instead of storing them.  Usage: ExchangeEnergy.apply(phi, grid, prec).
    """

    @staticmethod
    def forward(ctx, phi, grid, prec):
        phi = phi.contiguous()
        e = exchange_energy(phi, grid, prec)
        ctx.save_for_backward(phi)
        ctx.grid = grid
        ctx.prec = prec
        return e

    @staticmethod
    def backward(ctx, gbar):
        (phi,) = ctx.saved_tensors
        gb = gbar.detach().to(torch.float64).reshape(1).contiguous()
        g = exchange_energy_grad(phi, ctx.grid, ctx.prec, gbar=gb)
        return g, None, None
