"""ctypes binding of libsgmres.so (the gfx950 sketched GMRES library).

Argument marshalling only: every computation runs in the HIP kernels behind
the C ABI declared in include/sgmres.h.  PyTorch supplies device memory and the
current HIP stream.  There is no CPU fallback: if the library is missing or a
tensor is not on the GPU, the call raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgmres.so")

OK = 0
NOT_CONVERGED = 1
FLAG_KAPPA_TRUNC = 1
FLAG_BREAKDOWN = 2
BASIS_ARNOLDI = 0
BASIS_CHEBYSHEV = 1
PATH_ARNOLDI_3BAR = 1
PATH_ARNOLDI_HALO = 2
PATH_CHEBYSHEV = 3
PATH_PART_SPLIT = 4
PATH_STREAM = 5
PATH_MULTI = 6
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16_BASIS = 2
_PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16": PREC_BF16_BASIS}
ERRORS = {
    -1: "SGMRES_EINVAL (bad argument)",
    -2: "SGMRES_ECSR (malformed CSR)",
    -3: "SGMRES_ENOMEM (allocation failed)",
    -4: "SGMRES_EHIP (HIP runtime error)",
    -5: "SGMRES_ENONFINITE (NaN/Inf encountered)",
    -6: "SGMRES_ETIMEOUT (grid barrier wait limit)",
}


class SGMRESError(RuntimeError):
    def __init__(self, fn: str, rc: int):
        super().__init__(f"{fn} failed: {ERRORS.get(rc, rc)}")
        self.rc = rc


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("d_eff_last", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("relres", ctypes.c_double),
        ("rest_est", ctypes.c_double),
        ("kappa_est", ctypes.c_double),
        ("t_residual_ms", ctypes.c_double),
        ("t_basis_ms", ctypes.c_double),
        ("t_lsq_ms", ctypes.c_double),
        ("t_combine_ms", ctypes.c_double),
        ("phase_us", ctypes.c_double * 8),
        ("path", ctypes.c_int32),
        ("launch_block", ctypes.c_int32),
        ("launch_rows", ctypes.c_int32),
        ("launch_grid", ctypes.c_int32),
        ("t_sketch_ms", ctypes.c_double),
        ("cheb_box", ctypes.c_double * 3),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("zeta", ctypes.c_int32),
        ("kappa_max", ctypes.c_double),
        ("transposed", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("barrier_mode", ctypes.c_int32),
        ("spmv_mode", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("cheb_c", ctypes.c_double),
        ("cheb_dx", ctypes.c_double),
        ("cheb_dy", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("batch_eager", ctypes.c_int32),
        ("halo_off", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("stream_state", ctypes.c_int32),
    ]


class _System(ctypes.Structure):
    _fields_ = [("A", _CSR), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class _BatchResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("relres", ctypes.c_double),
    ]


_LIB = None


def lib():
    """Load libsgmres.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
    P = ctypes.POINTER
    L.sgmres_solve.argtypes = [P(_CSR), vp, vp, i32, i32, i32, u64, dbl, i32, P(_Info), vp]
    L.sgmres_solve_transposed.argtypes = L.sgmres_solve.argtypes
    L.sgmres_solve_ex.argtypes = [P(_CSR), vp, vp, i32, i32, i32, u64, dbl, i32, P(_Options), P(_Info), vp]
    L.sgmres_sketch_pattern.argtypes = [u64, u32, i64, i64, i32, i32, vp, vp, vp]
    L.sgmres_sketch_apply.argtypes = [i64, vp, u64, u32, i32, i32, vp, vp]
    L.sgmres_sketch_apply_noalloc.argtypes = [i64, vp, u64, u32, i32, i32, vp, vp]
    L.sgmres_residual.argtypes = [P(_CSR), vp, vp, vp, P(dbl), vp]
    L.sgmres_chebyshev_box.argtypes = [P(_CSR), vp, i32, vp, vp, P(i32), vp]
    L.sgmres_hessenberg_eigenvalues.argtypes = [i32, vp, i32, vp, vp]
    L.sgmres_arnoldi_cycle.argtypes = [P(_CSR), vp, i32, i32, i32, i32, u64, u32, vp, i64, vp, vp, vp, vp,
                                       P(i32), P(i32), vp]
    L.sgmres_solve_batched.argtypes = [i32, P(_System), i32, i32, i32, u64, dbl, i32, P(_Options),
                                       P(_BatchResult), vp]
    L.sgmres_chebyshev_cycle.argtypes = [P(_CSR), vp, i32, i32, i32, u64, u32, dbl, dbl, dbl, vp, i64, vp, vp,
                                         vp, vp, vp]
    L.sgmres_sketched_lsq.argtypes = [i32, i32, vp, vp, dbl, vp, P(i32), P(dbl), P(dbl), P(i32), vp]
    L.sgmres_basis_combine.argtypes = [i64, i32, vp, i64, vp, vp, vp]
    L.sgmres_csr_transpose.argtypes = [P(_CSR), vp, vp, vp, vp]
    L.sgmres_csr_outer_grad.argtypes = [P(_CSR), vp, vp, dbl, vp, vp]
    L.sgmres_plan_create.argtypes = [P(_CSR), i32, ctypes.POINTER(vp), vp]
    L.sgmres_plan_destroy.argtypes = [vp]
    L.sgmres_solve_plan.argtypes = [vp, vp, vp, i32, i32, i32, u64, dbl, i32, P(_Options), P(_Info), vp]
    L.sgmres_release_workspace.argtypes = []
    L.sgmres_release_workspace.restype = None
    L.sgmres_version.argtypes = []
    L.sgmres_version.restype = ctypes.c_char_p
    for name in ("sgmres_solve", "sgmres_solve_transposed", "sgmres_solve_ex", "sgmres_sketch_pattern",
                 "sgmres_plan_create", "sgmres_plan_destroy", "sgmres_solve_plan",
                 "sgmres_sketch_apply", "sgmres_sketch_apply_noalloc", "sgmres_residual", "sgmres_arnoldi_cycle", "sgmres_sketched_lsq",
                 "sgmres_basis_combine", "sgmres_csr_transpose", "sgmres_csr_outer_grad"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


@dataclasses.dataclass
class DeviceCSR:
    """CSR matrix whose arrays are torch tensors on a GPU."""

    n: int
    row_ptr: torch.Tensor  # int32[n+1]
    col_idx: torch.Tensor  # int32[nnz]
    val: torch.Tensor  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @classmethod
    def from_host(cls, A, device="cuda") -> "DeviceCSR":
        """Upload a host CSR (anything with n, row_ptr, col_idx, val arrays)."""
        return cls(
            n=int(A.n),
            row_ptr=torch.as_tensor(A.row_ptr, dtype=torch.int32).to(device),
            col_idx=torch.as_tensor(A.col_idx, dtype=torch.int32).to(device),
            val=torch.as_tensor(A.val, dtype=torch.float64).to(device),
        )

    def _c(self) -> _CSR:
        for t in (self.row_ptr, self.col_idx, self.val):
            _check_dev(t)
        if self.row_ptr.dtype != torch.int32 or self.col_idx.dtype != torch.int32:
            raise TypeError("row_ptr / col_idx must be int32")
        if self.val.dtype != torch.float64:
            raise TypeError("val must be float64")
        if self.row_ptr.numel() != self.n + 1:
            raise ValueError("row_ptr must have n+1 entries")
        return _CSR(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())


def _check_dev(t: torch.Tensor, dtype=None, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} entries, needs {numel}")
    return t


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _info(i: _Info) -> dict:
    return dict(cycles=i.cycles, steps=i.steps, d_eff_last=i.d_eff_last, flags=i.flags, relres=i.relres,
                rest_est=i.rest_est, kappa_est=i.kappa_est, t_residual_ms=i.t_residual_ms,
                t_basis_ms=i.t_basis_ms, t_lsq_ms=i.t_lsq_ms, t_combine_ms=i.t_combine_ms,
                phase_us=list(i.phase_us), path=i.path, launch_block=i.launch_block,
                launch_rows=i.launch_rows, launch_grid=i.launch_grid, t_sketch_ms=i.t_sketch_ms,
                cheb_box=tuple(i.cheb_box))


def _raise(fn, rc):
    if rc < 0:
        raise SGMRESError(fn, rc)
    return rc


def sgmres_solve(A: DeviceCSR, b, x, d, k, s, seed=0, tol=1e-10, restarts=100, *, zeta=8, kappa_max=1e14,
                 transposed=False, block_size=0, rows_per_thread=0, profile=False, barrier_mode=0,
                 spmv_mode=0, cheb_box=None, precision="fp64", halo_off=False, path=0, stream_state=0,
                 plan=None, stream=None):
    """Restarted sGMRES on A x = b (or A^T x = b); x is updated in place.

    cheb_box=(c, dx, dy) selects the Chebyshev basis for a spectrum inside
    [c - dx, c + dx] x [-dy, dy] (k is then unused), cheb_box="auto" the
    Chebyshev basis with the box estimated from a short Arnoldi pass on b
    (sgmres_chebyshev_box; reported in info["cheb_box"]); None selects
    k-truncated Arnoldi.  precision: "fp64", "fp32" (basis cycles in FP32) or "bf16" (FP32
    arithmetic, basis stored in bfloat16); the residual, least squares and x stay
    FP64, so restarting refines to FP64 accuracy.  halo_off=True keeps three grid
    barriers per truncated-Arnoldi step (the default uses two when few
    nonzeros reach outside their block; results are bit-identical).  path:
    0 (automatic), PATH_STREAM or PATH_PART_SPLIT to force the kernel used for
    systems beyond the resident capacity; stream_state: 0 auto, 1 registers,
    2 HBM buffer (streaming path).  plan: a Plan of A (its copies of A and A^T
    are reused instead of being rebuilt; A may then be None).  Returns (rc,
    info) with rc SGMRES_OK (0) or SGMRES_NOT_CONVERGED (1); raises SGMRESError
    on the negative error codes."""
    n = plan.A.n if plan is not None else A.n
    _check_dev(b, torch.float64, n)
    _check_dev(x, torch.float64, n)
    info = _Info()
    if isinstance(cheb_box, str):
        if cheb_box != "auto":
            raise ValueError("cheb_box: (c, dx, dy), 'auto' or None")
        cheb_box = (0.0, 0.0, 0.0)
    basis, (cc, cdx, cdy) = (0, (0.0, 0.0, 0.0)) if cheb_box is None else (1, tuple(float(t) for t in cheb_box))
    prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opts = _Options(zeta, kappa_max, 1 if transposed else 0, block_size, rows_per_thread, 1 if profile else 0,
                    barrier_mode, spmv_mode, basis, cc, cdx, cdy, prec, 0, 1 if halo_off else 0, path,
                    stream_state)
    if plan is not None:
        rc = lib().sgmres_solve_plan(plan.handle, b.data_ptr(), x.data_ptr(), d, k, s, seed, tol, restarts,
                                     ctypes.byref(opts), ctypes.byref(info), _stream(stream))
        return _raise("sgmres_solve_plan", rc), _info(info)
    rc = lib().sgmres_solve_ex(ctypes.byref(A._c()), b.data_ptr(), x.data_ptr(), d, k, s, seed, tol, restarts,
                               ctypes.byref(opts), ctypes.byref(info), _stream(stream))
    return _raise("sgmres_solve", rc), _info(info)


class Plan:
    """A matrix's set-up on the GPU (sgmres_plan_create): validated CSR, the
    sliced ELL copy of A (and of A^T with transpose=True; FP32 value copies
    with fp32=True), reused by every sgmres_solve(..., plan=...).  Keeps a
    reference to A's tensors; call close() (or use as a context manager) to
    free the device copies."""

    PLAN_TRANSPOSE = 1
    PLAN_FP32 = 2

    def __init__(self, A: "DeviceCSR", transpose: bool = False, fp32: bool = False, stream=None):
        self.A = A
        self.handle = None
        h = ctypes.c_void_p()
        flags = (self.PLAN_TRANSPOSE if transpose else 0) | (self.PLAN_FP32 if fp32 else 0)
        rc = lib().sgmres_plan_create(ctypes.byref(A._c()), flags, ctypes.byref(h), _stream(stream))
        _raise("sgmres_plan_create", rc)
        self.handle = h

    def close(self):
        if self.handle is not None:
            lib().sgmres_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sgmres_solve_batched(systems, d, k, s, seed=0, tol=1e-10, restarts=100, *, zeta=8, kappa_max=1e14,
                         precision="fp64", block_size=0, rows_per_thread=0, eager=False, path=0, stream=None):
    """Restarted sGMRES on many independent systems in one launch per cycle.

    systems: list of (DeviceCSR A, b, x) with b, x float64 GPU tensors (x is the
    initial guess, updated in place); several systems may share one A.  Returns
    (rc, results) with rc SGMRES_OK when all converged, SGMRES_NOT_CONVERGED
    otherwise, and one dict per system (status, cycles, steps, flags, relres).
    Systems sharing one DeviceCSR (n >= 65,536) are solved as blocks of up to
    32 right-hand sides by the streaming kernel; the other systems below 2^19
    rows run several to a resident basis launch (PATH_MULTI; rows_per_thread
    2 or 4, default 4).  path=PATH_PART_SPLIT keeps every system on the
    part-split kernel instead; path=PATH_MULTI requires the multi-system
    launch."""
    arr = (_System * max(len(systems), 1))()
    keep = []
    for i, (A, b, x) in enumerate(systems):
        _check_dev(b, torch.float64, A.n)
        _check_dev(x, torch.float64, A.n)
        c = A._c()
        keep.append(c)
        arr[i] = _System(c, b.data_ptr(), x.data_ptr())
    res = (_BatchResult * max(len(systems), 1))()
    prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opts = _Options(zeta, kappa_max, 0, block_size, rows_per_thread, 0, 0, 0, 0, 0.0, 0.0, 0.0, prec,
                    1 if eager else 0, 0, path, 0)
    rc = lib().sgmres_solve_batched(len(systems), arr, d, k, s, seed, tol, restarts, ctypes.byref(opts), res,
                                    _stream(stream))
    _raise("sgmres_solve_batched", rc)
    out = [dict(status=r.status, cycles=r.cycles, steps=r.steps, flags=r.flags, relres=r.relres)
           for r in res[: len(systems)]]
    return rc, out


def sgmres_chebyshev_box(A: DeviceCSR, r, m=20, stream=None):
    """Spectral box (c, dx, dy) for the Chebyshev basis from m + 1 Arnoldi
    steps on r (Section 4.4), and the Ritz values it is built from (a complex
    numpy array; shorter than m when the Krylov space of r is invariant)."""
    _check_dev(r, torch.float64, A.n)
    box = (ctypes.c_double * 3)()
    ritz = (ctypes.c_double * (2 * max(m, 1)))()
    nr = ctypes.c_int(0)
    rc = lib().sgmres_chebyshev_box(ctypes.byref(A._c()), r.data_ptr(), m, box, ritz, ctypes.byref(nr),
                                    _stream(stream))
    _raise("sgmres_chebyshev_box", rc)
    k = nr.value
    return (box[0], box[1], box[2]), np.array(ritz[:k]) + 1j * np.array(ritz[m:m + k])


def hessenberg_eigenvalues(H):
    """Eigenvalues of an upper Hessenberg matrix (host numpy array) by the
    library's double-shift QR iteration (entries below the subdiagonal are
    ignored)."""
    H = np.asfortranarray(np.asarray(H, dtype=np.float64))
    m = H.shape[0]
    if H.ndim != 2 or H.shape[1] != m:
        raise ValueError("H must be square")
    wr, wi = np.zeros(m), np.zeros(m)
    rc = lib().sgmres_hessenberg_eigenvalues(m, H.ctypes.data, m, wr.ctypes.data, wi.ctypes.data)
    _raise("sgmres_hessenberg_eigenvalues", rc)
    return wr + 1j * wi


def sgmres_solve_transposed(A: DeviceCSR, b, x, d, k, s, seed=0, tol=1e-10, restarts=100, stream=None):
    """Restarted sGMRES on A^T x = b through the dedicated entry point."""
    _check_dev(b, torch.float64, A.n)
    _check_dev(x, torch.float64, A.n)
    info = _Info()
    rc = lib().sgmres_solve_transposed(ctypes.byref(A._c()), b.data_ptr(), x.data_ptr(), d, k, s, seed, tol,
                                       restarts, ctypes.byref(info), _stream(stream))
    return _raise("sgmres_solve_transposed", rc), _info(info)


def sgmres_sketch_pattern(seed, cycle, i0, count, s, zeta, device="cuda", stream=None):
    """Rows (int32[count, zeta]) and signs (int8[count, zeta]) of sketch columns i0.. on the GPU."""
    rows = torch.empty((max(count, 1), zeta), dtype=torch.int32, device=device)
    signs = torch.empty((max(count, 1), zeta), dtype=torch.int8, device=device)
    rc = lib().sgmres_sketch_pattern(seed, cycle, i0, count, s, zeta, rows.data_ptr(), signs.data_ptr(),
                                     _stream(stream))
    _raise("sgmres_sketch_pattern", rc)
    return rows[:count], signs[:count]


def sgmres_sketch_apply(v, seed, cycle, s, zeta, stream=None):
    """g = S v on the GPU."""
    _check_dev(v, torch.float64)
    g = torch.empty(s, dtype=torch.float64, device=v.device)
    rc = lib().sgmres_sketch_apply(v.numel(), v.data_ptr(), seed, cycle, s, zeta, g.data_ptr(), _stream(stream))
    _raise("sgmres_sketch_apply", rc)
    return g


def sgmres_sketch_apply_noalloc(v, g, seed, cycle, s, zeta, stream=None):
    """g = S v into the caller's g (s float64 entries), with no allocation in
    the library; only enqueued on the stream."""
    _check_dev(v, torch.float64)
    _check_dev(g, torch.float64, s)
    rc = lib().sgmres_sketch_apply_noalloc(v.numel(), v.data_ptr(), seed, cycle, s, zeta, g.data_ptr(),
                                           _stream(stream))
    _raise("sgmres_sketch_apply_noalloc", rc)
    return g


def sgmres_residual(A: DeviceCSR, f, x, stream=None):
    """(r, |r|) with r = f - A x on the GPU."""
    _check_dev(f, torch.float64, A.n)
    _check_dev(x, torch.float64, A.n)
    r = torch.empty(A.n, dtype=torch.float64, device=f.device)
    nrm = ctypes.c_double(0)
    rc = lib().sgmres_residual(ctypes.byref(A._c()), f.data_ptr(), x.data_ptr(), r.data_ptr(), ctypes.byref(nrm),
                               _stream(stream))
    _raise("sgmres_residual", rc)
    return r, nrm.value


def sgmres_arnoldi_cycle(A: DeviceCSR, r, d, k, s, zeta=8, seed=0, cycle=0, stream=None):
    """One basis + sketch cycle; returns dict of GPU tensors (B n x d, SB, SAB s x d,
    H (k+1) x d, g) plus dc and flags."""
    _check_dev(r, torch.float64, A.n)
    dev = r.device
    B = torch.empty((d, A.n), dtype=torch.float64, device=dev)  # column-major n x d
    SB = torch.zeros((d, s), dtype=torch.float64, device=dev)
    SAB = torch.zeros((d, s), dtype=torch.float64, device=dev)
    H = torch.zeros((d, k + 1), dtype=torch.float64, device=dev)
    g = torch.empty(s, dtype=torch.float64, device=dev)
    dc = ctypes.c_int(0)
    flags = ctypes.c_int(0)
    rc = lib().sgmres_arnoldi_cycle(ctypes.byref(A._c()), r.data_ptr(), d, k, s, zeta, seed, cycle, B.data_ptr(),
                                    A.n, SB.data_ptr(), SAB.data_ptr(), H.data_ptr(), g.data_ptr(),
                                    ctypes.byref(dc), ctypes.byref(flags), _stream(stream))
    _raise("sgmres_arnoldi_cycle", rc)
    return dict(B=B.T, SB=SB.T, SAB=SAB.T, H=H.T, g=g, dc=dc.value, flags=flags.value)


def sgmres_chebyshev_cycle(A: DeviceCSR, r, d, s, c, dx, dy, zeta=8, seed=0, cycle=0, stream=None):
    """One Chebyshev-basis + sketch cycle; returns dict of GPU tensors: B (n x d,
    unnormalised recurrence vectors), colnorm (d), SB, SAB (s x d, of the
    normalised columns) and g."""
    _check_dev(r, torch.float64, A.n)
    dev = r.device
    B = torch.empty((d, A.n), dtype=torch.float64, device=dev)
    SB = torch.zeros((d, s), dtype=torch.float64, device=dev)
    SAB = torch.zeros((d, s), dtype=torch.float64, device=dev)
    cn = torch.empty(d, dtype=torch.float64, device=dev)
    g = torch.empty(s, dtype=torch.float64, device=dev)
    rc = lib().sgmres_chebyshev_cycle(ctypes.byref(A._c()), r.data_ptr(), d, s, zeta, seed, cycle, c, dx, dy,
                                      B.data_ptr(), A.n, SB.data_ptr(), SAB.data_ptr(), cn.data_ptr(), g.data_ptr(),
                                      _stream(stream))
    _raise("sgmres_chebyshev_cycle", rc)
    return dict(B=B.T, colnorm=cn, SB=SB.T, SAB=SAB.T, g=g)


def sgmres_sketched_lsq(SAB, g, kappa_max=1e14, stream=None):
    """Sketched LS on the GPU.  SAB: (s, dc) tensor (any layout), g: (s,).  Returns a dict."""
    s, dc = SAB.shape
    C = SAB.T.contiguous().clone()  # column-major storage, overwritten by the factorisation
    gg = g.contiguous().clone()
    _check_dev(C, torch.float64)
    _check_dev(gg, torch.float64, s)
    y = torch.zeros(max(dc, 1), dtype=torch.float64, device=C.device)
    d_eff = ctypes.c_int(0)
    rest = ctypes.c_double(0)
    kap = ctypes.c_double(0)
    flags = ctypes.c_int(0)
    rc = lib().sgmres_sketched_lsq(s, dc, C.data_ptr(), gg.data_ptr(), kappa_max, y.data_ptr(), ctypes.byref(d_eff),
                                   ctypes.byref(rest), ctypes.byref(kap), ctypes.byref(flags), _stream(stream))
    _raise("sgmres_sketched_lsq", rc)
    de = d_eff.value
    return dict(y=y[:de], d_eff=de, rest=rest.value, kappa=kap.value, flags=flags.value,
                T=torch.triu(C.T[:dc, :dc]), QTg=gg)


def sgmres_basis_combine(B, y, x, stream=None):
    """x <- x + B[:, :len(y)] y in place; B is an (n, d) tensor with column-major storage."""
    n = x.numel()
    _check_dev(x, torch.float64)
    d_eff = int(y.numel())
    Bc = B.T  # (d, n) row-major view of a column-major (n, d)
    if not Bc.is_contiguous():
        Bc = Bc.contiguous()
    yy = y.contiguous()
    rc = lib().sgmres_basis_combine(n, d_eff, Bc.data_ptr(), n, yy.data_ptr() if d_eff else None, x.data_ptr(),
                                    _stream(stream))
    _raise("sgmres_basis_combine", rc)
    return x


def sgmres_csr_transpose(A: DeviceCSR, stream=None) -> DeviceCSR:
    """CSR of A^T built on the GPU."""
    dev = A.val.device
    trp = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    tci = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    tv = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev)
    rc = lib().sgmres_csr_transpose(ctypes.byref(A._c()), trp.data_ptr(), tci.data_ptr(), tv.data_ptr(),
                                    _stream(stream))
    _raise("sgmres_csr_transpose", rc)
    return DeviceCSR(A.n, trp, tci[: A.nnz], tv[: A.nnz])


def sgmres_csr_outer_grad(A: DeviceCSR, u, v, alpha=-1.0, stream=None):
    """Values alpha * u[i] * v[j] on A's pattern (gradient of a solve w.r.t. A)."""
    _check_dev(u, torch.float64, A.n)
    _check_dev(v, torch.float64, A.n)
    dval = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=u.device)
    rc = lib().sgmres_csr_outer_grad(ctypes.byref(A._c()), u.data_ptr(), v.data_ptr(), alpha, dval.data_ptr(),
                                     _stream(stream))
    _raise("sgmres_csr_outer_grad", rc)
    return dval[: A.nnz]


def sgmres_release_workspace():
    lib().sgmres_release_workspace()


def sgmres_version() -> str:
    return lib().sgmres_version().decode()
