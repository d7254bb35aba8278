"""Python binding of libdpm with the names of the C ABI; torch tensors carry device memory.

Every function marshals tensors to device pointers and calls the library: the arithmetic of
every step runs in the HIP kernels.  Tensors must be CUDA (HIP) tensors, contiguous, FP64
unless stated.  Workspaces are allocated through torch's caching allocator.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L

PRECISIONS = {"fp64": L.DPM_FP64, "fp32": L.DPM_FP32, "bf16x3": L.DPM_BF16X3,
              "fp64_gemm": L.DPM_FP64_GEMM}


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev(t: torch.Tensor, name: str, dtype=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def grid(n: int, h: float, sigma: float = 0.0, x0: float = 0.0) -> L.Grid:
    return L.Grid(int(n), float(h), float(sigma), float(x0))


SWEEPS = {"auto": L.DPM_SWEEPS_AUTO, "axis": L.DPM_SWEEPS_AXIS, "plane": L.DPM_SWEEPS_PLANE,
          "split": L.DPM_SWEEPS_SPLIT}


def opts(prec: str = "fp64", io_fp64: bool = True, rtol: float = 1e-10, max_refine: int = 0,
         rhs_chunk: int = 0, sweeps: str = "auto") -> L.Opts:
    return L.Opts(PRECISIONS[prec], 1 if io_fp64 else 0, float(rtol), int(max_refine),
                  int(rhs_chunk), None, 0, SWEEPS[sweeps])


def workspace_size(g: L.Grid, nrhs: int, o: L.Opts) -> int:
    lib = L.load()
    nb = C.c_size_t(0)
    L.check(lib.dpm_workspace_size(C.byref(g), int(nrhs), C.byref(o), C.byref(nb)))
    return int(nb.value)


def rhs_chunk(g: L.Grid, nrhs: int, o: L.Opts) -> int:
    """Right-hand sides per sweep launch for a solve of nrhs right-hand sides."""
    c = C.c_int32(0)
    L.check(L.load().dpm_rhs_chunk(C.byref(g), int(nrhs), C.byref(o), C.byref(c)))
    return int(c.value)


def prepare(n: int) -> None:
    L.check(L.load().dpm_prepare(int(n)))


def aux_solve_batched(b: torch.Tensor, sigma: float, h: float, prec: str = "fp64",
                      rtol: float = 1e-10, max_refine: int = 0, out: torch.Tensor | None = None,
                      workspace: torch.Tensor | None = None, stream=None, info: bool = False,
                      rhs_chunk: int = 0, sweeps: str = "auto"):
    """Solve (sigma I - Lap_h) u = b for b of shape (nrhs, n, n, n) (or (n, n, n)).

    Returns u (and a dpm_info dict when info=True; that synchronises the stream).
    """
    lib = L.load()
    single = b.dim() == 3
    bb = b.unsqueeze(0) if single else b
    if bb.dim() != 4 or not (bb.shape[1] == bb.shape[2] == bb.shape[3]):
        raise ValueError("b must have shape (nrhs, n, n, n) or (n, n, n)")
    nrhs, n = int(bb.shape[0]), int(bb.shape[1])
    io_fp64 = bb.dtype == torch.float64
    if not io_fp64 and bb.dtype != torch.float32:
        raise ValueError("b must be float64 or float32")
    if out is None:
        out = torch.empty_like(bb)
    uu = out.view(bb.shape) if out.dim() == 3 else out
    g = grid(n, h, sigma)
    o = opts(prec, io_fp64, rtol, max_refine, rhs_chunk, sweeps)
    nbytes = workspace_size(g, nrhs, o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=bb.device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    inf = L.Info()
    st = lib.aux_solve_batched(C.byref(g), nrhs, C.c_void_p(_dev(bb, "b")),
                               C.c_void_p(_dev(uu, "u", bb.dtype)), C.byref(o),
                               C.c_void_p(_stream(stream)), C.byref(inf) if info else None)
    L.check(st)
    res = out if not single else out.view(n, n, n)
    if info:
        return res, {"refine_iters": inf.refine_iters, "est_rel_err": inf.est_rel_err}
    return res


def aux_solve_batched_noalloc(b: torch.Tensor, sigma: float, h: float, prec: str = "fp64",
                              rtol: float = 1e-10, max_refine: int = 0,
                              out: torch.Tensor | None = None, stream=None, info: bool = False,
                              rhs_chunk: int = 0, sweeps: str = "auto"):
    """aux_solve_batched through the entry point that allocates nothing on the device: no
    workspace is passed, the library's static device scratch is used.  `out` must be given by a
    caller that cannot allocate either (here a new tensor is made when it is None).  The size's
    tables must have been built first (prepare(n))."""
    lib = L.load()
    single = b.dim() == 3
    bb = b.unsqueeze(0) if single else b
    if bb.dim() != 4 or not (bb.shape[1] == bb.shape[2] == bb.shape[3]):
        raise ValueError("b must have shape (nrhs, n, n, n) or (n, n, n)")
    nrhs, n = int(bb.shape[0]), int(bb.shape[1])
    io_fp64 = bb.dtype == torch.float64
    if not io_fp64 and bb.dtype != torch.float32:
        raise ValueError("b must be float64 or float32")
    if out is None:
        out = torch.empty_like(bb)
    uu = out.view(bb.shape) if out.dim() == 3 else out
    g = grid(n, h, sigma)
    o = opts(prec, io_fp64, rtol, max_refine, rhs_chunk, sweeps)
    inf = L.Info()
    st = lib.aux_solve_batched_noalloc(C.byref(g), nrhs, C.c_void_p(_dev(bb, "b")),
                                       C.c_void_p(_dev(uu, "u", bb.dtype)), C.byref(o),
                                       C.c_void_p(_stream(stream)), C.byref(inf) if info else None)
    L.check(st)
    res = out if not single else out.view(n, n, n)
    if info:
        return res, {"refine_iters": inf.refine_iters, "est_rel_err": inf.est_rel_err}
    return res


SWEEP_NAMES = {L.DPM_SWEEPS_AXIS: "axis", L.DPM_SWEEPS_PLANE: "plane", L.DPM_SWEEPS_SPLIT: "split"}
LSQ_METHOD_NAMES = {0: "none", 1: "cholesky_qr2", 2: "householder", 3: "householder_truncated"}


def autotune(b: torch.Tensor, sigma: float, h: float, prec: str = "fp64", rtol: float = 1e-10,
             max_refine: int = 0, reps: int = 3, out: torch.Tensor | None = None,
             stream=None, sweeps: str = "auto") -> dict:
    """Time the batched solve of b (nrhs, n, n, n) at each candidate launch width (right-hand
    sides per sweep launch) and sweep layout, then the z pass's columns per block at the best
    pair, and record the fastest shape for this device, size and precision; later solves with
    rhs_chunk = 0 / sweeps = "auto" use it.  Returns {"widths", "sweeps", "zcols", "ms", "best",
    "best_sweeps", "best_zcols"}, with ms the best time per batched solve and zcols 0 for the
    default z tile.  u (out, or a new tensor) receives the solution.  Synchronises the stream."""
    lib = L.load()
    if b.dim() != 4 or not (b.shape[1] == b.shape[2] == b.shape[3]):
        raise ValueError("b must have shape (nrhs, n, n, n)")
    nrhs, n = int(b.shape[0]), int(b.shape[1])
    io_fp64 = b.dtype == torch.float64
    if not io_fp64 and b.dtype != torch.float32:
        raise ValueError("b must be float64 or float32")
    if out is None:
        out = torch.empty_like(b)
    g = grid(n, h, sigma)
    # a workspace for the widest candidate fits every narrower one, in every layout the size has
    # (the split layout's separator planes included where it exists)
    nbytes = workspace_size(g, nrhs, opts(prec, io_fp64, rtol, max_refine, min(16, nrhs)))
    try:
        nbytes = max(nbytes, workspace_size(g, nrhs, opts(prec, io_fp64, rtol, max_refine,
                                                          min(16, nrhs), "split")))
    except L.DPMError:
        pass
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=b.device)
    o = opts(prec, io_fp64, rtol, max_refine, 0, sweeps)
    o.workspace = C.c_void_p(ws.data_ptr())
    o.workspace_bytes = ws.numel()
    nc = L.DPM_TUNE_MAX_CANDIDATES
    widths = (C.c_int32 * nc)()
    lays = (C.c_int32 * nc)()
    zc = (C.c_int32 * nc)()
    ms = (C.c_double * nc)()
    count, best, best_l, best_z = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
    L.check(lib.dpm_autotune(C.byref(g), nrhs, C.byref(o), C.c_void_p(_dev(b, "b")),
                             C.c_void_p(_dev(out, "u", b.dtype)), int(reps),
                             C.c_void_p(_stream(stream)), widths, lays, zc, ms, C.byref(count),
                             C.byref(best), C.byref(best_l), C.byref(best_z)))
    k = count.value
    return {"widths": list(widths[:k]), "sweeps": [SWEEP_NAMES[v] for v in lays[:k]],
            "zcols": list(zc[:k]), "ms": list(ms[:k]), "best": best.value,
            "best_sweeps": SWEEP_NAMES[best_l.value], "best_zcols": best_z.value}


def autotune_reset() -> None:
    """Forget every recorded launch shape (solves go back to the library's defaults)."""
    L.load().dpm_autotune_reset()


def aux_solve_batched_sigma(b: torch.Tensor, sigmas, h: float, prec: str = "fp64",
                            rtol: float = 1e-10, max_refine: int = 0,
                            out: torch.Tensor | None = None,
                            workspace: torch.Tensor | None = None, stream=None,
                            rhs_chunk: int = 0, sweeps: str = "auto"):
    """Batched solve with one shift per right-hand side: b (nrhs, n, n, n), sigmas (nrhs,)."""
    lib = L.load()
    nrhs, n = int(b.shape[0]), int(b.shape[1])
    sig = (C.c_double * nrhs)(*[float(x) for x in sigmas])
    if len(sig) != nrhs:
        raise ValueError("one sigma per right-hand side")
    io_fp64 = b.dtype == torch.float64
    out = torch.empty_like(b) if out is None else out
    g = grid(n, h, 0.0)
    o = opts(prec, io_fp64, rtol, max_refine, rhs_chunk, sweeps)
    nbytes = workspace_size(g, nrhs, o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=b.device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    L.check(lib.aux_solve_batched_sigma(C.byref(g), nrhs, sig, C.c_void_p(_dev(b, "b")),
                                        C.c_void_p(_dev(out, "u", b.dtype)), C.byref(o),
                                        C.c_void_p(_stream(stream)), None))
    return out


def aux_solve(b: torch.Tensor, sigma: float, h: float, **kw):
    """Single right-hand side (n, n, n); see aux_solve_batched."""
    if b.dim() != 3:
        raise ValueError("aux_solve takes one (n, n, n) right-hand side")
    return aux_solve_batched(b, sigma, h, **kw)


def geometry(kind: str = "sphere", center=(0.0, 0.0, 0.0), axes=(1.0, 1.0, 1.0)) -> L.Geometry:
    k = {"sphere": 0, "ellipsoid": 1}[kind]
    ax = (axes, axes, axes) if isinstance(axes, (int, float)) else tuple(axes)
    if len(ax) == 1:
        ax = (ax[0], ax[0], ax[0])
    return L.Geometry(k, (C.c_double * 3)(*center), (C.c_double * 3)(*ax))


def classify(n: int, h: float, x0: float, geo: L.Geometry, device="cuda", stream=None):
    """M+ mask (uint8, n^3) of the nodes strictly inside the geometry."""
    m = torch.empty((n, n, n), dtype=torch.uint8, device=device)
    g = grid(n, h, 0.0, x0)
    L.check(L.load().dpm_classify(C.byref(g), C.byref(geo), C.c_void_p(m.data_ptr()),
                                  C.c_void_p(_stream(stream))))
    return m


def gamma_points(m_plus: torch.Tensor, h: float = 1.0, x0: float = 0.0, stream=None):
    """(idx int32, is_in uint8) of the discrete grid boundary, ascending linear index."""
    lib = L.load()
    n = int(m_plus.shape[-1])
    g = grid(n, h, 0.0, x0)
    ng, ngi = C.c_int32(0), C.c_int32(0)
    mp = C.c_void_p(_dev(m_plus, "m_plus", torch.uint8))
    L.check(lib.dpm_gamma_points(C.byref(g), mp, C.byref(ng), C.byref(ngi), None, None,
                                 C.c_void_p(_stream(stream))))
    idx = torch.empty(ng.value, dtype=torch.int32, device=m_plus.device)
    is_in = torch.empty(ng.value, dtype=torch.uint8, device=m_plus.device)
    L.check(lib.dpm_gamma_points(C.byref(g), mp, C.byref(ng), C.byref(ngi),
                                 C.c_void_p(idx.data_ptr()), C.c_void_p(is_in.data_ptr()),
                                 C.c_void_p(_stream(stream))))
    return idx, is_in


def basis(n: int, h: float, x0: float, geo: L.Geometry, idx: torch.Tensor, lmax: int,
          beta: int = 1, stream=None):
    """(basis (n_basis, n_gamma) FP64, d (n_gamma) FP64) of the spectral densities."""
    ng = int(idx.numel())
    nb = (beta + 1) * (lmax + 1) ** 2
    B = torch.empty((nb, ng), dtype=torch.float64, device=idx.device)
    d = torch.empty(ng, dtype=torch.float64, device=idx.device)
    g = grid(n, h, 0.0, x0)
    L.check(L.load().dpm_basis(C.byref(g), C.byref(geo), ng, C.c_void_p(_dev(idx, "idx", torch.int32)),
                               int(lmax), int(beta), C.c_void_p(B.data_ptr()),
                               C.c_void_p(d.data_ptr()), C.c_void_p(_stream(stream))))
    return B, d


def basis_zonal(n: int, h: float, x0: float, geo: L.Geometry, idx: torch.Tensor, mmax: int,
                beta: int = 0, stream=None):
    """(basis ((beta + 1)(mmax + 1), n_gamma) FP64, d (n_gamma) FP64): Legendre P_nu(cos theta)."""
    ng = int(idx.numel())
    nb = (beta + 1) * (mmax + 1)
    B = torch.empty((nb, ng), dtype=torch.float64, device=idx.device)
    d = torch.empty(ng, dtype=torch.float64, device=idx.device)
    g = grid(n, h, 0.0, x0)
    L.check(L.load().dpm_basis_zonal(C.byref(g), C.byref(geo), ng,
                                     C.c_void_p(_dev(idx, "idx", torch.int32)), int(mmax),
                                     int(beta), C.c_void_p(B.data_ptr()),
                                     C.c_void_p(d.data_ptr()), C.c_void_p(_stream(stream))))
    return B, d


class BEP:
    """Owner of a dpm_bep handle (boundary matrix, QR, point sets); released on close()."""

    def __init__(self, ptr: int, n: int, h: float, sigma: float, x0: float, device):
        self.ptr = ptr
        self.n, self.h, self.sigma, self.x0 = n, h, sigma, x0
        self.device = device
        ng, ngi, nb = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        rmin, rmax = C.c_double(0), C.c_double(0)
        L.check(L.load().dpm_bep_info(C.c_void_p(ptr), C.byref(ng), C.byref(ngi), C.byref(nb),
                                      C.byref(rmin), C.byref(rmax)))
        self.n_gamma, self.n_gamma_in, self.n_basis = ng.value, ngi.value, nb.value
        self.rdiag = (rmin.value, rmax.value)

    def rebuild_workspace_size(self) -> int:
        nb = C.c_size_t(0)
        L.check(L.load().dpm_bep_rebuild_workspace_size(C.c_void_p(self.ptr), C.byref(nb)))
        return int(nb.value)

    def device_bytes(self) -> int:
        """Device memory the handle holds."""
        nb = C.c_size_t(0)
        L.check(L.load().dpm_bep_device_bytes(C.c_void_p(self.ptr), C.byref(nb)))
        return int(nb.value)

    def rebuild(self, sigma: float, stream=None, workspace: torch.Tensor | None = None) -> None:
        """Step 4b: the matrix, its QR and the least-squares operator again at a new sigma, with
        the scratch in `workspace` (allocated here through torch when not given)."""
        nbytes = self.rebuild_workspace_size()
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        L.check(L.load().dpm_bep_rebuild(C.c_void_p(self.ptr), float(sigma),
                                         C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         C.c_void_p(_stream(stream))))
        self.sigma = float(sigma)
        self._refresh_rdiag()

    def _refresh_rdiag(self):
        rmin, rmax = C.c_double(0), C.c_double(0)
        L.check(L.load().dpm_bep_info(C.c_void_p(self.ptr), None, None, None, C.byref(rmin),
                                      C.byref(rmax)))
        self.rdiag = (rmin.value, rmax.value)

    def lsq_method(self) -> str:
        """The QR behind the least-squares operator of the last build or rebuild:
        "cholesky_qr2" or "householder"."""
        m = C.c_int32(0)
        L.check(L.load().dpm_bep_lsq_method(C.c_void_p(self.ptr), C.byref(m)))
        return LSQ_METHOD_NAMES[m.value]

    def close(self):
        if self.ptr:
            L.load().dpm_bep_destroy(C.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_boundary_matrix(m_plus: torch.Tensor, basis_mat: torch.Tensor, n: int, h: float,
                          sigma: float, x0: float = 0.0, prec: str = "fp64", rtol: float = 1e-10,
                          max_refine: int = 0, rhs_chunk: int = 0, return_A: bool = False,
                          stream=None):
    """Step 2: the reduced-BEP matrix of the densities `basis_mat` (n_basis x n_gamma) and its QR.

    Returns a BEP handle (and A, |gamma_in| x n_basis, when return_A)."""
    lib = L.load()
    g = grid(n, h, sigma, x0)
    o = opts(prec, True, rtol, max_refine, rhs_chunk)
    nb = int(basis_mat.shape[0])
    out = C.c_void_p(0)
    A = None
    if return_A:
        # |gamma_in| is known only after classification: count first
        _, is_in = gamma_points(m_plus, h, x0, stream)
        A = torch.empty((nb, int(is_in.sum().item())), dtype=torch.float64, device=m_plus.device)
    L.check(lib.dpm_build_boundary_matrix(
        C.byref(g), C.c_void_p(_dev(m_plus, "m_plus", torch.uint8)), nb,
        C.c_void_p(_dev(basis_mat, "basis", torch.float64)), C.byref(o),
        C.c_void_p(_stream(stream)), C.byref(out), C.c_void_p(A.data_ptr()) if A is not None else None))
    bep = BEP(out.value, n, h, sigma, x0, m_plus.device)
    if return_A:
        return bep, A.t()   # column-major storage -> (|gamma_in|, n_basis) view
    return bep


class DD:
    """Owner of a dpm_dd handle: the two subdomains of the domain decomposition (Case 1), their
    point sets and densities, and the QR of the coupled reduced BEPs; released on close()."""

    def __init__(self, ptr: int, params: L.DDParams, device):
        self.ptr = ptr
        self.params = params
        self.device = device
        self.sigma = params.grid1.sigma
        self.n = (params.grid1.n, params.grid2.n)
        ng, ngi, nr = (C.c_int32 * 2)(), (C.c_int32 * 2)(), (C.c_int32 * 2)()
        nc, rmin, rmax = C.c_int32(0), C.c_double(0), C.c_double(0)
        L.check(L.load().dpm_dd_info(C.c_void_p(ptr), ng, ngi, nr, C.byref(nc), C.byref(rmin),
                                     C.byref(rmax)))
        self.n_gamma, self.n_gamma_in, self.n_rows = tuple(ng), tuple(ngi), tuple(nr)
        self.n_cols = nc.value
        self.rdiag = (rmin.value, rmax.value)

    def lsq_info(self) -> dict:
        """rcond of the coupled least squares, the numerical rank of the coupled matrix, the
        smallest kept singular value over the largest (truncated least squares only) and the QR
        used ("cholesky_qr2", "householder" or "householder_truncated")."""
        rc, rk, sm, me = C.c_double(0), C.c_int32(0), C.c_double(0), C.c_int32(0)
        lib = L.load()
        L.check(lib.dpm_dd_lsq_info(C.c_void_p(self.ptr), C.byref(rc), C.byref(rk), C.byref(sm)))
        L.check(lib.dpm_dd_lsq_method(C.c_void_p(self.ptr), C.byref(me)))
        return {"rcond": rc.value, "rank": rk.value, "smin_ratio": sm.value,
                "method": LSQ_METHOD_NAMES[me.value]}

    def masks(self, l: int, stream=None):
        """(M+, N+) of subdomain l as uint8 volumes."""
        n = self.n[l]
        mp = torch.empty((n, n, n), dtype=torch.uint8, device=self.device)
        np_ = torch.empty_like(mp)
        L.check(L.load().dpm_dd_masks(C.c_void_p(self.ptr), l, C.c_void_p(mp.data_ptr()),
                                      C.c_void_p(np_.data_ptr()), C.c_void_p(_stream(stream))))
        return mp, np_

    def gauss_state(self, l: int, amp: float, rate: float, center=(0.0, 0.0, 0.0), stream=None):
        n = self.n[l]
        out = torch.empty((n, n, n), dtype=torch.float64, device=self.device)
        L.check(L.load().dpm_dd_gauss_state(C.c_void_p(self.ptr), l, float(amp), float(rate),
                                            (C.c_double * 3)(*center), C.c_void_p(out.data_ptr()),
                                            C.c_void_p(_stream(stream))))
        return out

    def workspace_size(self, o: L.Opts) -> int:
        nb = C.c_size_t(0)
        L.check(L.load().dpm_dd_step_workspace_size(C.c_void_p(self.ptr), C.byref(o), C.byref(nb)))
        return int(nb.value)

    def rebuild_workspace_size(self) -> int:
        nb = C.c_size_t(0)
        L.check(L.load().dpm_dd_rebuild_workspace_size(C.c_void_p(self.ptr), C.byref(nb)))
        return int(nb.value)

    def run_workspace_size(self, o: L.Opts) -> int:
        nb = C.c_size_t(0)
        L.check(L.load().dpm_dd_run_workspace_size(C.c_void_p(self.ptr), C.byref(o), C.byref(nb)))
        return int(nb.value)

    def rebuild(self, sigma: float, stream=None, workspace: torch.Tensor | None = None) -> None:
        """Step 4b: both subdomains' columns and the coupled QR again at a new sigma, with the
        scratch in `workspace` (allocated here through torch when not given)."""
        nbytes = self.rebuild_workspace_size()
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        L.check(L.load().dpm_dd_rebuild(C.c_void_p(self.ptr), float(sigma),
                                        C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                        C.c_void_p(_stream(stream))))
        self.sigma = float(sigma)
        self._refresh()

    def _refresh(self):
        rmin, rmax = C.c_double(0), C.c_double(0)
        L.check(L.load().dpm_dd_info(C.c_void_p(self.ptr), None, None, None, None, C.byref(rmin),
                                     C.byref(rmax)))
        self.rdiag = (rmin.value, rmax.value)

    def close(self):
        if self.ptr:
            L.load().dpm_dd_destroy(C.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dd_params(n1: int, h1: float, x01: float, n2: int, h2: float, x02: float, sigma: float,
              r_z: float, r_gamma: float, r_split: float, m_gamma: int, beta: int, m_z: int,
              center=(0.0, 0.0, 0.0)) -> L.DDParams:
    return L.DDParams(grid(n1, h1, sigma, x01), grid(n2, h2, sigma, x02), (C.c_double * 3)(*center),
                      float(r_z), float(r_gamma), float(r_split), int(m_gamma), int(beta), int(m_z))


def dd2_params(n1: int, h1: float, x01: float, origin1, n2: int, h2: float, x02: float, origin2,
               sigma: float, r_gamma: float, q_z: float, r_z: float, eps_layers: float,
               m_gamma: int, beta: int, m_z: int, rcond: float = 0.0) -> L.DD2Params:
    return L.DD2Params(grid(n1, h1, sigma, x01), grid(n2, h2, sigma, x02),
                       (C.c_double * 3)(*origin1), (C.c_double * 3)(*origin2), float(r_gamma),
                       float(q_z), float(r_z), float(eps_layers), int(m_gamma), int(beta), int(m_z),
                       float(rcond))


def dd_build(params, prec: str = "fp64", device="cuda", return_A: bool = False, stream=None,
             rtol: float = 1e-10, max_refine: int = 0):
    """Step 2 of the domain decomposition (Case 1 for DDParams, Case 2 for DD2Params): both
    subdomains' columns, the stacked matrix and its QR.  Returns a DD handle (and the stacked
    matrix, rows x n_cols, when return_A: the row count is known only after a first build, so
    that case builds twice)."""
    lib = L.load()
    fn = lib.dpm_dd2_build if isinstance(params, L.DD2Params) else lib.dpm_dd_build
    o = opts(prec, True, rtol, max_refine)
    out = C.c_void_p(0)
    L.check(fn(C.byref(params), C.byref(o), C.c_void_p(_stream(stream)), C.byref(out), None))
    dd = DD(out.value, params, torch.device(device))
    if not return_A:
        return dd
    rows = sum(dd.n_rows)
    dd.close()
    A = torch.empty((dd.n_cols, rows), dtype=torch.float64, device=device)
    out = C.c_void_p(0)
    L.check(fn(C.byref(params), C.byref(o), C.c_void_p(_stream(stream)), C.byref(out),
               C.c_void_p(A.data_ptr())))
    return DD(out.value, params, torch.device(device)), A.t()


def dd_step(dd: DD, dt: float, chi: float, state, out=None, prec: str = "fp64",
            workspace: torch.Tensor | None = None, stream=None, rtol: float = 1e-10,
            max_refine: int = 0):
    """One step on both subdomains; state = (rho_1, c_1, rho_2, c_2); returns the new four."""
    for v, n in zip(state, (dd.n[0], dd.n[0], dd.n[1], dd.n[1])):
        if v.numel() != n ** 3:
            raise ValueError(f"state volumes must hold {dd.n[0]}^3, {dd.n[0]}^3, {dd.n[1]}^3, "
                             f"{dd.n[1]}^3 values")
    if out is not None and any(a.numel() != b.numel() for a, b in zip(out, state)):
        raise ValueError("out volumes must match the state volumes")
    o = opts(prec, True, rtol, max_refine)
    nbytes = dd.workspace_size(o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=state[0].device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    out = [torch.empty_like(v) for v in state] if out is None else out
    names = ("rho_1", "c_1", "rho_2", "c_2")
    pin = (C.c_void_p * 4)(*[_dev(v, k, torch.float64) for v, k in zip(state, names)])
    pout = (C.c_void_p * 4)(*[_dev(v, k + "_out", torch.float64) for v, k in zip(out, names)])
    L.check(L.load().dpm_dd_step(C.c_void_p(dd.ptr), float(dt), float(chi), pin, pout,
                                 C.byref(o), C.c_void_p(_stream(stream))))
    return tuple(out)


class DDStepper:
    """Graph-captured fixed-dt time loop on the decomposed domain, state updated in place."""

    def __init__(self, dd: DD, dt: float, chi: float, state, prec: str = "fp64",
                 rtol: float = 1e-10, max_refine: int = 0, workspace: torch.Tensor | None = None):
        for v, n in zip(state, (dd.n[0], dd.n[0], dd.n[1], dd.n[1])):
            if v.numel() != n ** 3:
                raise ValueError("state volumes must match the subdomains' meshes")
        o = opts(prec, True, rtol, max_refine)
        nbytes = dd.workspace_size(o)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=state[0].device)
        o.workspace = C.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel()
        # the graph keeps raw pointers: hold the buffers for its lifetime
        self.dd, self.state, self.workspace = dd, list(state), workspace
        names = ("rho_1", "c_1", "rho_2", "c_2")
        pst = (C.c_void_p * 4)(*[_dev(v, k, torch.float64) for v, k in zip(state, names)])
        out = C.c_void_p(0)
        L.check(L.load().dpm_dd_stepper_create(C.c_void_p(dd.ptr), float(dt), float(chi), pst,
                                               C.byref(o), C.byref(out)))
        self.ptr = out.value

    def run(self, nsteps: int, stream=None) -> None:
        L.check(L.load().dpm_dd_stepper_run(C.c_void_p(self.ptr), int(nsteps),
                                            C.c_void_p(_stream(stream))))

    def close(self):
        if self.ptr:
            L.load().dpm_dd_stepper_destroy(C.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dd_run(dd: DD, chi: float, state, t_final: float, rho_cap: float = float("inf"),
           max_steps: int = 1000, prec: str = "fp64", workspace: torch.Tensor | None = None,
           stream=None, rtol: float = 1e-10, max_refine: int = 0,
           rho_jump_cap: float = 0.0) -> dict:
    """Steps 3-8 on the decomposed domain, state = (rho_1, c_1, rho_2, c_2) in place, from
    dt = 1/dd.sigma; the run summary as for run()."""
    for v, n in zip(state, (dd.n[0], dd.n[0], dd.n[1], dd.n[1])):
        if v.numel() != n ** 3:
            raise ValueError(f"state volumes must hold {dd.n[0]}^3, {dd.n[0]}^3, {dd.n[1]}^3, "
                             f"{dd.n[1]}^3 values")
    o = opts(prec, True, rtol, max_refine)
    nbytes = dd.run_workspace_size(o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=state[0].device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    p = L.RunParams(float(chi), float(t_final), float(rho_cap), int(max_steps), float(rho_jump_cap))
    info = L.RunInfo()
    dts = (C.c_double * max(int(max_steps), 1))()
    rbs = (C.c_uint8 * max(int(max_steps), 1))()
    names = ("rho_1", "c_1", "rho_2", "c_2")
    pst = (C.c_void_p * 4)(*[_dev(v, k, torch.float64) for v, k in zip(state, names)])
    L.check(L.load().dpm_dd_run(C.c_void_p(dd.ptr), C.byref(p), pst, C.byref(o),
                                C.c_void_p(_stream(stream)), C.byref(info), dts, rbs))
    k = info.steps
    if info.rebuilds > 0:
        dd.sigma = 1.0 / info.dt
        dd._refresh()
    return {"steps": k, "rebuilds": info.rebuilds, "stop": L.RUN_STOPS[info.stop], "t": info.t,
            "dt": info.dt, "rho_max": info.rho_max, "grad_max": info.grad_max,
            "dt_hist": [dts[i] for i in range(k)], "rebuilt": [bool(rbs[i]) for i in range(k)]}


def diagnostics(bep: BEP, rho: torch.Tensor, c: torch.Tensor, stream=None) -> torch.Tensor:
    """(max |rho| over M+, second moment, free energy) as a device tensor of 3 FP64."""
    out = torch.empty(3, dtype=torch.float64, device=rho.device)
    ws = torch.empty(L.DPM_DIAG_WORKSPACE_BYTES, dtype=torch.uint8, device=rho.device)
    n3 = bep.n ** 3
    if rho.numel() != n3 or c.numel() != n3:
        raise ValueError(f"rho and c must hold {bep.n}^3 values")
    L.check(L.load().dpm_diagnostics(C.c_void_p(bep.ptr), C.c_void_p(_dev(rho, "rho", torch.float64)),
                                     C.c_void_p(_dev(c, "c", torch.float64)),
                                     C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     ws.numel(), C.c_void_p(_stream(stream))))
    return out


def dd_diagnostics(dd: DD, state, stream=None) -> torch.Tensor:
    """The same over both subdomains, state = (rho_1, c_1, rho_2, c_2)."""
    for v, n in zip(state, (dd.n[0], dd.n[0], dd.n[1], dd.n[1])):
        if v.numel() != n ** 3:
            raise ValueError("state volumes must match the subdomains' meshes")
    out = torch.empty(3, dtype=torch.float64, device=state[0].device)
    ws = torch.empty(L.DPM_DIAG_WORKSPACE_BYTES, dtype=torch.uint8, device=state[0].device)
    names = ("rho_1", "c_1", "rho_2", "c_2")
    pst = (C.c_void_p * 4)(*[_dev(v, k, torch.float64) for v, k in zip(state, names)])
    L.check(L.load().dpm_dd_diagnostics(C.c_void_p(dd.ptr), pst, C.c_void_p(out.data_ptr()),
                                        C.c_void_p(ws.data_ptr()), ws.numel(),
                                        C.c_void_p(_stream(stream))))
    return out


def bep_solve(bep: BEP, g: torch.Tensor, stream=None) -> torch.Tensor:
    """Least-squares coefficients for g of shape (nvec, |gamma_in|)."""
    gg = g.unsqueeze(0) if g.dim() == 1 else g
    Cc = torch.empty((gg.shape[0], bep.n_basis), dtype=torch.float64, device=gg.device)
    L.check(L.load().dpm_bep_solve(C.c_void_p(bep.ptr), int(gg.shape[0]),
                                   C.c_void_p(_dev(gg, "g", torch.float64)),
                                   C.c_void_p(Cc.data_ptr()), C.c_void_p(_stream(stream))))
    return Cc[0] if g.dim() == 1 else Cc


def run_workspace_size(bep: BEP, o: L.Opts) -> int:
    """Bytes of dpm_run's workspace: step workspace, scan area and rebuild scratch."""
    nb = C.c_size_t(0)
    L.check(L.load().dpm_run_workspace_size(C.c_void_p(bep.ptr), C.byref(o), C.byref(nb)))
    return int(nb.value)


def step_workspace_size(bep: BEP, o: L.Opts) -> int:
    nb = C.c_size_t(0)
    L.check(L.load().dpm_step_workspace_size(C.c_void_p(bep.ptr), C.byref(o), C.byref(nb)))
    return int(nb.value)


def dpm_step(bep: BEP, dt: float, chi: float, rho: torch.Tensor, c: torch.Tensor,
             rho_out: torch.Tensor | None = None, c_out: torch.Tensor | None = None,
             prec: str = "fp64", rtol: float = 1e-10, max_refine: int = 0,
             workspace: torch.Tensor | None = None, stream=None, info: bool = False,
             sweeps: str = "auto"):
    """Steps 4a-7 for (rho, c) on N+; returns (rho_new, c_new)."""
    lib = L.load()
    o = opts(prec, True, rtol, max_refine, 0, sweeps)
    nbytes = step_workspace_size(bep, o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=rho.device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    rho_out = torch.empty_like(rho) if rho_out is None else rho_out
    c_out = torch.empty_like(c) if c_out is None else c_out
    inf = L.Info()
    L.check(lib.dpm_step(C.c_void_p(bep.ptr), float(dt), float(chi),
                         C.c_void_p(_dev(rho, "rho", torch.float64)),
                         C.c_void_p(_dev(c, "c", torch.float64)),
                         C.c_void_p(_dev(rho_out, "rho_out", torch.float64)),
                         C.c_void_p(_dev(c_out, "c_out", torch.float64)), C.byref(o),
                         C.c_void_p(_stream(stream)), C.byref(inf) if info else None))
    if info:
        return rho_out, c_out, {"refine_iters": inf.refine_iters, "est_rel_err": inf.est_rel_err}
    return rho_out, c_out


class Stepper:
    """Graph-captured time loop: dpm_step on (rho, c) in place, replayed on demand."""

    def __init__(self, bep: BEP, dt: float, chi: float, rho: torch.Tensor, c: torch.Tensor,
                 prec: str = "fp64", rtol: float = 1e-10, max_refine: int = 0,
                 workspace: torch.Tensor | None = None, stream=None):
        lib = L.load()
        o = opts(prec, True, rtol, max_refine)
        nbytes = step_workspace_size(bep, o)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=rho.device)
        o.workspace = C.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel()
        # the handle keeps raw pointers: hold the tensors for its lifetime
        self.bep, self.rho, self.c, self.workspace = bep, rho, c, workspace
        out = C.c_void_p(0)
        L.check(lib.dpm_stepper_create(C.c_void_p(bep.ptr), float(dt), float(chi),
                                       C.c_void_p(_dev(rho, "rho", torch.float64)),
                                       C.c_void_p(_dev(c, "c", torch.float64)), C.byref(o),
                                       C.c_void_p(_stream(stream)), C.byref(out)))
        self.ptr = out.value

    def run(self, nsteps: int, stream=None) -> None:
        L.check(L.load().dpm_stepper_run(C.c_void_p(self.ptr), int(nsteps),
                                         C.c_void_p(_stream(stream))))

    def first_nonfinite(self, stream=None) -> int:
        v = C.c_int32(0)
        L.check(L.load().dpm_stepper_first_nonfinite(C.c_void_p(self.ptr),
                                                     C.c_void_p(_stream(stream)), C.byref(v)))
        return int(v.value)

    def close(self):
        if self.ptr:
            L.load().dpm_stepper_destroy(C.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cfl_scan(bep: BEP, rho: torch.Tensor, c: torch.Tensor, stream=None) -> torch.Tensor:
    """Device tensor [max |grad_h c| over the faces of M+ nodes, max |rho| over M+]."""
    out = torch.empty(2, dtype=torch.float64, device=rho.device)
    L.check(L.load().dpm_cfl_scan(C.c_void_p(bep.ptr), C.c_void_p(_dev(rho, "rho", torch.float64)),
                                  C.c_void_p(_dev(c, "c", torch.float64)),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(_stream(stream))))
    return out


def run(bep: BEP, chi: float, rho: torch.Tensor, c: torch.Tensor, t_final: float,
        rho_cap: float = float("inf"), max_steps: int = 1000, prec: str = "fp64",
        rtol: float = 1e-10, max_refine: int = 0, workspace: torch.Tensor | None = None,
        stream=None, rho_jump_cap: float = 0.0) -> dict:
    """Steps 3-8: the adaptive time loop on (rho, c) in place, from dt = 1/bep.sigma.

    Returns the run summary with the per-step dt and rebuild flags; the handle then holds the
    matrix of the last dt (bep.sigma is updated)."""
    lib = L.load()
    o = opts(prec, True, rtol, max_refine)
    nbytes = run_workspace_size(bep, o)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=rho.device)
    o.workspace = C.c_void_p(workspace.data_ptr())
    o.workspace_bytes = workspace.numel()
    p = L.RunParams(float(chi), float(t_final), float(rho_cap), int(max_steps), float(rho_jump_cap))
    info = L.RunInfo()
    dts = (C.c_double * max(int(max_steps), 1))()
    rbs = (C.c_uint8 * max(int(max_steps), 1))()
    L.check(lib.dpm_run(C.c_void_p(bep.ptr), C.byref(p), C.c_void_p(_dev(rho, "rho", torch.float64)),
                        C.c_void_p(_dev(c, "c", torch.float64)), C.byref(o),
                        C.c_void_p(_stream(stream)), C.byref(info), dts, rbs))
    k = info.steps
    if info.rebuilds > 0:  # the library rebuilt at sigma = 1/dt (the same division)
        bep.sigma = 1.0 / info.dt
        bep._refresh_rdiag()
    return {"steps": k, "rebuilds": info.rebuilds, "stop": L.RUN_STOPS[info.stop], "t": info.t,
            "dt": info.dt, "rho_max": info.rho_max, "grad_max": info.grad_max,
            "dt_hist": [dts[i] for i in range(k)], "rebuilt": [bool(rbs[i]) for i in range(k)]}


def gauss_state(bep: BEP, geo: L.Geometry, amp: float, rate: float, center=(0.0, 0.0, 0.0),
                stream=None) -> torch.Tensor:
    """amp exp(-rate |x - center|^2) on M+, and at the projection onto Gamma on gamma."""
    out = torch.empty((bep.n, bep.n, bep.n), dtype=torch.float64, device=bep.device)
    c3 = (C.c_double * 3)(*center)
    L.check(L.load().dpm_gauss_state(C.c_void_p(bep.ptr), C.byref(geo), float(amp), float(rate),
                                     c3, C.c_void_p(out.data_ptr()), C.c_void_p(_stream(stream))))
    return out
