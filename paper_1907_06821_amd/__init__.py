"""paper_1907_06821_amd: folded-spectrum plane-wave eigensolver for MI355X (gfx950).

Thin ctypes binding over libpw.so (include/pw.h).  Every function here only
marshals arguments; all arithmetic runs in the library's HIP kernels.  torch is
used for device memory and streams.  If libpw.so is missing or cannot be
loaded, importing the compute entry points raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIBPATH = _HERE / "libpw.so"

PW_OK, PW_EINVAL, PW_ENOMEM, PW_EHIP, PW_ENOTPD, PW_ENOCONV, PW_ENAN, PW_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
PW_C128, PW_C64 = 0, 1
PW_PREP_C128, PW_PREP_C64, PW_PREP_C128_OTF = 1, 2, 4

_STATUS_NAMES = {0: "PW_OK", -1: "PW_EINVAL", -2: "PW_ENOMEM", -3: "PW_EHIP", -4: "PW_ENOTPD",
                 -5: "PW_ENOCONV", -6: "PW_ENAN", -7: "PW_EUNSUPPORTED"}

# names declared in include/pw.h (checked by the test-suite against the library's exports)
EXPORTS = ("pw_basis_size", "pw_basis_miller", "pw_ctx_create", "pw_ctx_destroy", "pw_ctx_get_info",
           "pw_ctx_kinetic", "pw_ctx_shells", "pw_hpsi", "pw_wave_to_grid", "pw_grid_to_wave",
           "pw_orthonormalize", "pw_cg_opts_default", "pw_folded_cg_solve", "pw_dense_eigh",
           "pw_dense_chol_inv", "pw_mlp_set", "pw_mlp_forward", "pw_mlp_harvest", "pw_mlp_work_bytes",
           "pw_mlp_loss_grad", "pw_mlp_adam", "pw_mlp_train", "pw_profile_begin",
           "pw_profile_end", "pw_last_error", "pw_batch_solve", "pw_ctx_autotune", "pw_ctx_fft_choose",
           "pw_lin_opts_default", "pw_folded_linear_solve", "pw_cheb_filter", "pw_chebfd_step",
           "pw_spectral_bounds", "pw_kinterp", "pw_ctx_set_otf_atoms", "pw_dense_eigh_noalloc")
PROF_KINDS = ("z_inverse", "xy_fft_v", "z_forward_kinetic", "projection", "back_projection", "block_rotate3",
              "block_gram", "block_rotate", "block_gram_herm")
PW_PROF_NKINDS = 9


class PwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class pw_cell(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("cell", C.c_double * 3), ("kpt", C.c_double * 3), ("ecut", C.c_double)]


class pw_potential(C.Structure):
    _fields_ = [("v_r", C.c_void_p), ("natom", C.c_int32), ("pos", C.POINTER(C.c_double)), ("nl", C.c_int32),
                ("sigma", C.c_double), ("d", C.POINTER(C.c_double))]


class pw_ctx_info(C.Structure):
    _fields_ = [("npw", C.c_int32), ("ncols", C.c_int32), ("nshell", C.c_int32), ("nproj", C.c_int32),
                ("grid", C.c_int32 * 3), ("max_bands", C.c_int32), ("device_bytes", C.c_int64),
                ("cols_bands", C.c_int32)]


class pw_cg_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("precond", C.c_int32), ("delta_e", C.c_double),
                ("precision", C.c_int32), ("check_every", C.c_int32), ("verbose", C.c_int32),
                ("mixed_switch", C.c_double), ("stall_checks", C.c_int32), ("snap_buf", C.c_void_p),
                ("snap_every", C.c_int32), ("snap_cap", C.c_int32), ("nconv", C.c_int32),
                ("batch_launch", C.c_int32), ("learned_stall", C.c_int32), ("recover", C.c_int32),
                ("fault_check", C.c_int32)]


class pw_lin_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("precond", C.c_int32), ("delta_e", C.c_double),
                ("check_every", C.c_int32), ("verbose", C.c_int32), ("use_graph", C.c_int32)]


class pw_lin_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("n_hpsi", C.c_int64), ("max_resid", C.c_double),
                ("seconds", C.c_double), ("n_hist", C.c_int32), ("hist", C.POINTER(C.c_double))]


class pw_fft_cand(C.Structure):
    _fields_ = [("pass_", C.c_int32), ("kind", C.c_int32), ("nthr", C.c_int32), ("sched", C.c_int32),
                ("nradix", C.c_int32), ("radix", C.c_int32 * 12), ("ms", C.c_double), ("chosen", C.c_int32)]


class pw_cg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("n_hpsi", C.c_int64), ("max_resid", C.c_double),
                ("seconds", C.c_double), ("n_hist", C.c_int32), ("hist", C.POINTER(C.c_double)),
                ("n_snap", C.c_int32), ("precond_switch_it", C.c_int32), ("recoveries", C.c_int32),
                ("fused", C.c_int32), ("ms", C.c_double * 4)]


_lib = None


def lib():
    """The loaded libpw.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not LIBPATH.exists():
            raise ImportError(f"{LIBPATH} is not built; run __graft_entry__.build() or "
                              "python -m paper_1907_06821_amd.csrc.build")
        L = C.CDLL(str(LIBPATH))
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "pw_basis_size": [C.POINTER(pw_cell), C.POINTER(i32)],
            "pw_basis_miller": [C.POINTER(pw_cell), C.POINTER(i32), i32],
            "pw_ctx_create": [C.POINTER(pw_cell), C.POINTER(pw_potential), i32, i32, vp, C.POINTER(vp)],
            "pw_ctx_destroy": [vp],
            "pw_ctx_get_info": [vp, C.POINTER(pw_ctx_info)],
            "pw_ctx_set_otf_atoms": [vp, i32],
            "pw_ctx_kinetic": [vp, C.POINTER(dbl)],
            "pw_ctx_shells": [vp, C.POINTER(i32), C.POINTER(dbl)],
            "pw_hpsi": [vp, i32, i32, vp, i64, vp, i64, dbl, vp],
            "pw_wave_to_grid": [vp, i32, i32, vp, i64, vp, vp],
            "pw_grid_to_wave": [vp, i32, i32, vp, vp, i64, vp],
            "pw_orthonormalize": [vp, i32, vp, i64, vp],
            "pw_folded_cg_solve": [vp, dbl, i32, vp, i64, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(pw_cg_opts),
                                   C.POINTER(pw_cg_stats), vp],
            "pw_dense_eigh": [i32, vp, i64, vp, vp, i32, dbl, C.POINTER(i32), vp],
            "pw_dense_eigh_noalloc": [i32, vp, i64, vp, vp, i32, dbl, C.POINTER(i32), vp],
            "pw_dense_chol_inv": [i32, vp, i64, vp, vp],
            "pw_mlp_set": [vp, vp],
            "pw_mlp_forward": [i32, i32, vp, vp, dbl, dbl, vp, vp, vp],
            "pw_mlp_harvest": [vp, dbl, i32, vp, vp, i64, dbl, dbl, vp, vp, vp],
            "pw_mlp_loss_grad": [i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, vp, i64, vp],
            "pw_mlp_adam": [vp, vp, vp, vp, i32, C.c_float, vp],
            "pw_mlp_train": [i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, vp, i32, i32, C.c_float,
                             C.POINTER(C.c_float), vp, i64, vp],
            "pw_profile_begin": [vp, i32],
            "pw_profile_end": [vp, C.POINTER(dbl), C.POINTER(i64)],
            "pw_batch_solve": [i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp],
            "pw_ctx_autotune": [vp, i32, i32, i32, vp, i32, C.POINTER(i32), vp],
            "pw_ctx_fft_choose": [vp, i32, vp],
            "pw_folded_linear_solve": [vp, dbl, i32, vp, i64, vp, i64, i32, vp, i64, C.POINTER(dbl),
                                       C.POINTER(dbl), C.POINTER(dbl), C.POINTER(pw_lin_opts),
                                       C.POINTER(pw_lin_stats), vp],
            "pw_cheb_filter": [vp, i32, vp, i64, vp, i64, dbl, dbl, i32, dbl, dbl, vp],
            "pw_chebfd_step": [vp, i32, vp, i64, dbl, dbl, i32, dbl, dbl, C.POINTER(dbl), C.POINTER(dbl), vp],
            "pw_spectral_bounds": [vp, vp, i32, C.POINTER(dbl), C.POINTER(dbl), vp],
            "pw_kinterp": [vp, vp, vp, dbl, i32, vp, i64, C.POINTER(dbl), vp, i64, C.POINTER(dbl), C.POINTER(dbl),
                           vp, i64, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.pw_mlp_work_bytes.argtypes = [i32, i32, i32]
        L.pw_mlp_work_bytes.restype = C.c_int64
        L.pw_cg_opts_default.argtypes = [C.POINTER(pw_cg_opts)]
        L.pw_cg_opts_default.restype = None
        L.pw_lin_opts_default.argtypes = [C.POINTER(pw_lin_opts)]
        L.pw_lin_opts_default.restype = None
        L.pw_last_error.argtypes = []
        L.pw_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != PW_OK:
        raise PwError(status, lib().pw_last_error().decode(errors="replace"))


def make_cell(grid, cell, ecut, kpt=(0.0, 0.0, 0.0)):
    c = pw_cell()
    for a in range(3):
        c.n[a] = int(grid[a])
        c.cell[a] = float(cell[a])
        c.kpt[a] = float(kpt[a])
    c.ecut = float(ecut)
    return c


def basis_miller(grid, cell, ecut, kpt=(0.0, 0.0, 0.0)):
    """Miller triples of the basis in coefficient order (host computation in the library)."""
    c = make_cell(grid, cell, ecut, kpt)
    n = C.c_int32()
    _check(lib().pw_basis_size(C.byref(c), C.byref(n)))
    out = np.empty((n.value, 3), dtype=np.int32)
    _check(lib().pw_basis_miller(C.byref(c), out.ctypes.data_as(C.POINTER(C.c_int32)), n.value))
    return out


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex128:
        return PW_C128
    if t.dtype == torch.complex64:
        return PW_C64
    raise TypeError(f"expected complex128 or complex64, got {t.dtype}")


def _check_block(t, npw):
    if not t.is_cuda:
        raise ValueError("blocks must live on the GPU")
    if t.dim() != 2 or t.stride(1) != 1 or t.stride(0) < npw or t.shape[1] != npw:
        raise ValueError(f"expected a [nb, {npw}] row-contiguous block, got shape {tuple(t.shape)} "
                         f"stride {t.stride()}")


class Context:
    """A pw_ctx: basis, tables and workspace of one problem on the current GPU.

    vgrid: float64 [N0, N1, N2] local potential samples (numpy or torch).
    pos, dproj: atom centres [natom, 3] (bohr) and KB strengths [natom * nl] (Ha).
    flags: PW_PREP_C128 and/or PW_PREP_C64, or PW_PREP_C128_OTF (complex128 without a stored
    projector table: rows generated per H psi)."""

    def __init__(self, grid, cell, ecut, vgrid, pos=None, nl=0, sigma=0.8, dproj=None, kpt=(0.0, 0.0, 0.0),
                 max_bands=128, flags=PW_PREP_C128, stream=None):
        import torch
        self._lib = lib()
        self.handle = C.c_void_p()
        self.cellc = make_cell(grid, cell, ecut, kpt)
        v = torch.as_tensor(np.ascontiguousarray(vgrid, dtype=np.float64)).to("cuda")
        if tuple(v.shape) != tuple(int(x) for x in grid):
            raise ValueError("vgrid shape does not match the grid")
        pot = pw_potential()
        pot.v_r = v.data_ptr()
        pos_np = np.ascontiguousarray(np.zeros((0, 3)) if pos is None else pos, dtype=np.float64)
        d_np = np.ascontiguousarray(np.zeros(0) if dproj is None else dproj, dtype=np.float64)
        pot.natom = int(pos_np.shape[0]) if nl else 0
        pot.pos = pos_np.ctypes.data_as(C.POINTER(C.c_double))
        pot.nl = int(nl)
        pot.sigma = float(sigma)
        pot.d = d_np.ctypes.data_as(C.POINTER(C.c_double))
        st = _stream_ptr(stream)
        _check(self._lib.pw_ctx_create(C.byref(self.cellc), C.byref(pot), int(max_bands), int(flags), st,
                                       C.byref(self.handle)))
        torch.cuda.current_stream().synchronize()
        info = pw_ctx_info()
        _check(self._lib.pw_ctx_get_info(self.handle, C.byref(info)))
        self.npw, self.ncols, self.nshell, self.nproj = info.npw, info.ncols, info.nshell, info.nproj
        self.cols_bands = info.cols_bands
        self.grid = tuple(int(x) for x in grid)
        self.max_bands = int(max_bands)

    @classmethod
    def from_problem(cls, prob, max_bands=None, flags=PW_PREP_C128, vgrid=None):
        return cls(prob.grid, prob.cell, prob.ecut, prob.vgrid() if vgrid is None else vgrid,
                   pos=prob.pos, nl=prob.nl, sigma=prob.sigma, dproj=prob.dproj, kpt=prob.kpt,
                   max_bands=max_bands or prob.nbands, flags=flags)

    def set_otf_atoms(self, atoms):
        """Atoms per chunk of the generated projector rows (PW_PREP_C128_OTF contexts)."""
        _check(self._lib.pw_ctx_set_otf_atoms(self.handle, int(atoms)))

    def info(self):
        info = pw_ctx_info()
        _check(self._lib.pw_ctx_get_info(self.handle, C.byref(info)))
        return {f: getattr(info, f) if f != "grid" else tuple(info.grid) for f, _ in pw_ctx_info._fields_}

    def kinetic(self):
        out = np.empty(self.npw)
        _check(self._lib.pw_ctx_kinetic(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def shells(self):
        sid = np.empty(self.npw, dtype=np.int32)
        st = np.empty(self.nshell)
        _check(self._lib.pw_ctx_shells(self.handle, sid.ctypes.data_as(C.POINTER(C.c_int32)),
                                       st.ctypes.data_as(C.POINTER(C.c_double))))
        return sid, st

    def close(self):
        if self.handle:
            _check(self._lib.pw_ctx_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hpsi(ctx, psi, shift=0.0, out=None, stream=None):
    """out = (H - shift) psi; complex128 -> FP64 path, complex64 -> mixed path."""
    import torch
    _check_block(psi, ctx.npw)
    if out is None:
        out = torch.empty_like(psi)
    _check_block(out, ctx.npw)
    _check(ctx._lib.pw_hpsi(ctx.handle, _dtype_code(psi), psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                            C.c_void_p(out.data_ptr()), out.stride(0), float(shift), _stream_ptr(stream)))
    return out


def wave_to_grid(ctx, psi, stream=None):
    import torch
    _check_block(psi, ctx.npw)
    out = torch.empty((psi.shape[0],) + ctx.grid, dtype=psi.dtype, device=psi.device)
    _check(ctx._lib.pw_wave_to_grid(ctx.handle, _dtype_code(psi), psi.shape[0], C.c_void_p(psi.data_ptr()),
                                    psi.stride(0), C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def grid_to_wave(ctx, grid, stream=None):
    import torch
    if tuple(grid.shape[1:]) != ctx.grid or not grid.is_contiguous():
        raise ValueError("grid must be a contiguous [nb, N0, N1, N2] tensor")
    out = torch.empty((grid.shape[0], ctx.npw), dtype=grid.dtype, device=grid.device)
    _check(ctx._lib.pw_grid_to_wave(ctx.handle, _dtype_code(grid), grid.shape[0], C.c_void_p(grid.data_ptr()),
                                    C.c_void_p(out.data_ptr()), out.stride(0), _stream_ptr(stream)))
    return out


def orthonormalize(ctx, psi, stream=None):
    """In-place Gram/Cholesky orthonormalisation of a complex128 block."""
    _check_block(psi, ctx.npw)
    _check(ctx._lib.pw_orthonormalize(ctx.handle, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                      _stream_ptr(stream)))
    return psi


def dense_eigh(a, key=0, ref=0.0, stream=None, noalloc=False):
    """Hermitian eigensolver on a [n, n] complex128 device matrix: (w, R, sweeps),
    rows of R are eigenvectors (w ordered by key: 0 ascending, 1 by |w - ref|).
    noalloc: call pw_dense_eigh_noalloc (library-held work memory, n <= 512)."""
    import torch
    n = a.shape[0]
    if a.dtype != torch.complex128 or not a.is_cuda or a.shape != (n, n) or a.stride(1) != 1:
        raise ValueError("expected a row-contiguous [n, n] complex128 CUDA tensor")
    w = torch.empty(n, dtype=torch.float64, device=a.device)
    r = torch.empty((n, n), dtype=torch.complex128, device=a.device)
    sw = C.c_int32()
    fn = lib().pw_dense_eigh_noalloc if noalloc else lib().pw_dense_eigh
    _check(fn(n, C.c_void_p(a.data_ptr()), a.stride(0), C.c_void_p(w.data_ptr()), C.c_void_p(r.data_ptr()),
              int(key), float(ref), C.byref(sw), _stream_ptr(stream)))
    return w, r, sw.value


def dense_chol_inv(s, stream=None):
    """T = conj(L^{-1}) with s = L L^H (complex128 device matrix)."""
    import torch
    n = s.shape[0]
    if s.dtype != torch.complex128 or not s.is_cuda or s.shape != (n, n) or s.stride(1) != 1:
        raise ValueError("expected a row-contiguous [n, n] complex128 CUDA tensor")
    t = torch.empty((n, n), dtype=torch.complex128, device=s.device)
    _check(lib().pw_dense_chol_inv(n, C.c_void_p(s.data_ptr()), s.stride(0), C.c_void_p(t.data_ptr()),
                                   _stream_ptr(stream)))
    return t


MLP_NPARAM = 4481


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _need(t, dtype, n=None):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or (n is not None and t.numel() != n):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor" + (f" of {n} elements" if n else ""))


def mlp_set(ctx, weights):
    """Install float32 network weights (device, MLP_NPARAM) for precond=2."""
    import torch
    _need(weights, torch.float32, MLP_NPARAM)
    _check(lib().pw_mlp_set(ctx.handle, _dptr(weights)))


def mlp_forward(shell_t, tband, e_ref, ecut, weights, stream=None):
    """f [nshell, nb] (float32) for device float64 shell_t [nshell], tband [nb]."""
    import torch
    _need(shell_t, torch.float64)
    _need(tband, torch.float64)
    _need(weights, torch.float32, MLP_NPARAM)
    f = torch.empty((shell_t.numel(), tband.numel()), dtype=torch.float32, device=shell_t.device)
    _check(lib().pw_mlp_forward(shell_t.numel(), tband.numel(), _dptr(shell_t), _dptr(tband), float(e_ref),
                                float(ecut), _dptr(weights), _dptr(f), _stream_ptr(stream)))
    return f


def mlp_harvest(ctx, e_ref, x_snap, x_conv, weight_delta=-1.0, delta_e=1.0, stream=None):
    """Training tables of one snapshot: (tabs [3, nshell, nb] float64, tband [nb]);
    K0 = M(G) with delta_e; weight_delta >= 0 weights shell s by
    (T_s - e_ref)^2 + weight_delta^2."""
    import torch
    _check_block(x_snap, ctx.npw)
    _check_block(x_conv, ctx.npw)
    nb = x_snap.shape[0]
    if x_conv.shape[0] != nb or x_snap.stride(0) != x_conv.stride(0):
        raise ValueError("x_snap and x_conv must have the same shape and stride")
    tabs = torch.empty((3, ctx.nshell, nb), dtype=torch.float64, device=x_snap.device)
    tband = torch.empty(nb, dtype=torch.float64, device=x_snap.device)
    _check(lib().pw_mlp_harvest(ctx.handle, float(e_ref), nb, _dptr(x_snap), _dptr(x_conv), x_snap.stride(0),
                                float(delta_e), float(weight_delta), _dptr(tabs), _dptr(tband),
                                _stream_ptr(stream)))
    return tabs, tband


def mlp_work_bytes(nshell, nb, nsnap):
    return int(lib().pw_mlp_work_bytes(nshell, nb, nsnap))


def mlp_loss_grad(shell_t, tband, e_ref, ecut, tabs, weights, stream=None):
    """(loss, grad) on device; tband [nsnap, nb], e_ref [nsnap], tabs [nsnap, 3, nshell, nb]."""
    import torch
    nsnap, nb = tband.shape
    ns = shell_t.numel()
    for t in (shell_t, tband, e_ref, tabs):
        _need(t, torch.float64)
    if tuple(tabs.shape) != (nsnap, 3, ns, nb) or e_ref.numel() != nsnap:
        raise ValueError("table shapes do not match")
    _need(weights, torch.float32, MLP_NPARAM)
    wb = mlp_work_bytes(ns, nb, nsnap)
    work = torch.empty(wb, dtype=torch.uint8, device=tabs.device)
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=tabs.device)
    loss = torch.empty(1, dtype=torch.float32, device=tabs.device)
    _check(lib().pw_mlp_loss_grad(ns, nb, nsnap, _dptr(shell_t), _dptr(tband), _dptr(e_ref), float(ecut),
                                  _dptr(tabs), _dptr(weights), _dptr(grad), _dptr(loss), _dptr(work), wb,
                                  _stream_ptr(stream)))
    return loss, grad


def mlp_adam(weights, grad, m, v, step, lr, stream=None):
    _check(lib().pw_mlp_adam(_dptr(weights), _dptr(grad), _dptr(m), _dptr(v), int(step), float(lr),
                             _stream_ptr(stream)))


def mlp_train(shell_t, tband, e_ref, ecut, tabs, weights, nsteps, lr=3e-3, m=None, v=None, step0=0, stream=None):
    """nsteps Adam steps on the device (weights updated in place); returns the loss history."""
    import torch
    nsnap, nb = tband.shape
    ns = shell_t.numel()
    for t in (shell_t, tband, e_ref, tabs):
        _need(t, torch.float64)
    _need(weights, torch.float32, MLP_NPARAM)
    dev = weights.device
    m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev) if m is None else m
    v = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=dev) if v is None else v
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=dev)
    wb = mlp_work_bytes(ns, nb, nsnap) + 4 * (nsteps + 64)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    hist = np.zeros(max(nsteps, 1), dtype=np.float32)
    _check(lib().pw_mlp_train(ns, nb, nsnap, _dptr(shell_t), _dptr(tband), _dptr(e_ref), float(ecut), _dptr(tabs),
                              _dptr(weights), _dptr(grad), _dptr(m), _dptr(v), int(step0), int(nsteps), float(lr),
                              hist.ctypes.data_as(C.POINTER(C.c_float)), _dptr(work), wb, _stream_ptr(stream)))
    return hist[:nsteps], m, v


def profile_begin(ctx, max_records=100000):
    _check(ctx._lib.pw_profile_begin(ctx.handle, int(max_records)))


def profile_end(ctx):
    """{stage kind: (total ms, launches)} for the launches since profile_begin."""
    ms = np.zeros(PW_PROF_NKINDS)
    n = np.zeros(PW_PROF_NKINDS, dtype=np.int64)
    _check(ctx._lib.pw_profile_end(ctx.handle, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                   n.ctypes.data_as(C.POINTER(C.c_int64))))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROF_KINDS)}


def cg_opts(**kw):
    o = pw_cg_opts()
    lib().pw_cg_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def folded_cg_solve(ctx, e_ref, psi, opts=None, hist_len=0, stream=None, raise_on_noconv=True, **kw):
    """Folded-spectrum PCG on the complex128 block psi (in: start, out: Ritz vectors).

    snapshots (optional): complex128 device tensor [cap, nb, npw] receiving the
    iterate every `snap_every` iterations.
    Returns (eig [nb] ascending, resid [nb], stats dict)."""
    _check_block(psi, ctx.npw)
    nb = psi.shape[0]
    snaps = kw.pop("snapshots", None)
    o = opts if opts is not None else cg_opts(**kw)
    if snaps is not None:
        import torch
        if (snaps.dtype != torch.complex128 or not snaps.is_cuda or not snaps.is_contiguous()
                or tuple(snaps.shape[1:]) != (nb, ctx.npw)):
            raise ValueError("snapshots must be a contiguous complex128 [cap, nb, npw] CUDA tensor")
        o.snap_buf = snaps.data_ptr()
        o.snap_cap = snaps.shape[0]
    eig = np.zeros(nb)
    res = np.zeros(nb)
    st = pw_cg_stats()
    hist = np.zeros((max(hist_len, 0), 2))
    st.n_hist = int(hist_len)
    st.hist = hist.ctypes.data_as(C.POINTER(C.c_double)) if hist_len else C.POINTER(C.c_double)()
    status = ctx._lib.pw_folded_cg_solve(ctx.handle, float(e_ref), nb, C.c_void_p(psi.data_ptr()), psi.stride(0),
                                         eig.ctypes.data_as(C.POINTER(C.c_double)),
                                         res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o), C.byref(st),
                                         _stream_ptr(stream))
    stats = dict(iters=st.iters, converged=bool(st.converged), n_hpsi=st.n_hpsi, max_resid=st.max_resid,
                 seconds=st.seconds, hist=hist[:st.n_hist].copy(), status=status, n_snap=st.n_snap,
                 precond_switch_it=st.precond_switch_it, recoveries=st.recoveries,
                 ms_setup=st.ms[0], ms_iters=st.ms[1], ms_checks=st.ms[2], ms_final=st.ms[3])
    if status != PW_OK and not (status == PW_ENOCONV and not raise_on_noconv):
        _check(status)
    return eig, res, stats


def lin_opts(**kw):
    o = pw_lin_opts()
    lib().pw_lin_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def folded_linear_solve(ctx, e, w, psi, phi=None, eps=None, delta=None, opts=None, hist_len=0, stream=None,
                        raise_on_noconv=True, **kw):
    """PCG on (H - E)^2 psi = (H - E) w for the complex128 sources w [nrhs, npw]
    (psi: in, start guess; out, solution).  precond=1 builds M' from the
    eigenpairs (phi [nev, npw] device, eps and delta host arrays [nev]).
    Returns (resid [nrhs], stats dict)."""
    import torch
    for t in (w, psi) + ((phi,) if phi is not None else ()):
        _check_block(t, ctx.npw)
        if t.dtype != torch.complex128:
            raise ValueError("the linear solve takes complex128 blocks")
    if tuple(w.shape) != tuple(psi.shape):
        raise ValueError("w and psi must have the same shape")
    nrhs = psi.shape[0]
    o = opts if opts is not None else lin_opts(**kw)
    nev, phi_ptr, ldphi = 0, None, 0
    eps_a = delta_a = None
    if phi is not None:
        nev, phi_ptr, ldphi = phi.shape[0], phi.data_ptr(), phi.stride(0)
        eps_a = np.ascontiguousarray(eps, dtype=np.float64)
        delta_a = np.ascontiguousarray(delta, dtype=np.float64)
        if eps_a.shape != (nev,) or delta_a.shape != (nev,):
            raise ValueError("eps and delta must have one entry per eigenvector")
    dp = C.POINTER(C.c_double)
    res = np.zeros(nrhs)
    st = pw_lin_stats()
    hist = np.zeros((max(hist_len, 0), 2))
    st.n_hist = int(hist_len)
    st.hist = hist.ctypes.data_as(dp) if hist_len else dp()
    status = ctx._lib.pw_folded_linear_solve(
        ctx.handle, float(e), nrhs, C.c_void_p(w.data_ptr()), w.stride(0), C.c_void_p(psi.data_ptr()),
        psi.stride(0), nev, C.c_void_p(phi_ptr), ldphi,
        eps_a.ctypes.data_as(dp) if eps_a is not None else dp(),
        delta_a.ctypes.data_as(dp) if delta_a is not None else dp(),
        res.ctypes.data_as(dp), C.byref(o), C.byref(st), _stream_ptr(stream))
    stats = dict(iters=st.iters, converged=bool(st.converged), n_hpsi=st.n_hpsi, max_resid=st.max_resid,
                 seconds=st.seconds, hist=hist[:st.n_hist].copy(), status=status)
    if status != PW_OK and not (status == PW_ENOCONV and not raise_on_noconv):
        _check(status)
    return res, stats


def _c128_block(t, npw):
    import torch
    _check_block(t, npw)
    if t.dtype != torch.complex128:
        raise ValueError("expected a complex128 block")


def cheb_filter(ctx, psi, e, half_width, degree, emin, emax, stream=None):
    """p(H) psi for the Chebyshev window filter of [e - w, e + w] (new tensor)."""
    import torch
    _c128_block(psi, ctx.npw)
    out = torch.empty_like(psi)
    _check(ctx._lib.pw_cheb_filter(ctx.handle, psi.shape[0], C.c_void_p(psi.data_ptr()), psi.stride(0),
                                   C.c_void_p(out.data_ptr()), out.stride(0), float(e), float(half_width),
                                   int(degree), float(emin), float(emax), _stream_ptr(stream)))
    return out


def chebfd_step(ctx, psi, e, half_width, degree, emin, emax, stream=None):
    """One ChebFD step in place on psi; returns (eig ascending, resid)."""
    _c128_block(psi, ctx.npw)
    nb = psi.shape[0]
    eig = np.zeros(nb)
    res = np.zeros(nb)
    dp = C.POINTER(C.c_double)
    _check(ctx._lib.pw_chebfd_step(ctx.handle, nb, C.c_void_p(psi.data_ptr()), psi.stride(0), float(e),
                                   float(half_width), int(degree), float(emin), float(emax),
                                   eig.ctypes.data_as(dp), res.ctypes.data_as(dp), _stream_ptr(stream)))
    return eig, res


def spectral_bounds(ctx, v0, steps=40, stream=None):
    """(emin, emax) estimate from `steps` Lanczos steps on H from v0 (complex128 [npw] on the GPU)."""
    import torch
    if not v0.is_cuda or v0.dtype != torch.complex128 or v0.numel() != ctx.npw or not v0.is_contiguous():
        raise ValueError("v0 must be a contiguous complex128 CUDA vector of npw entries")
    lo, hi = C.c_double(), C.c_double()
    _check(ctx._lib.pw_spectral_bounds(ctx.handle, C.c_void_p(v0.data_ptr()), int(steps), C.byref(lo), C.byref(hi),
                                       _stream_ptr(stream)))
    return lo.value, hi.value


def kinterp(ctx1, ctx2, ctxk, alpha, psi1, eps1, psi2, eps2, states=True, stream=None):
    """Energies at k = k2 + alpha (k1 - k2) interpolated from the eigenpairs at k1
    and k2 (complex128 blocks [n, npw] on each context's sphere); with states=True
    also the interpolated states on ctxk's sphere.  Returns (eps, psi_k or None)."""
    import torch
    _c128_block(psi1, ctx1.npw)
    _c128_block(psi2, ctx2.npw)
    n = psi1.shape[0]
    if psi2.shape[0] != n:
        raise ValueError("psi1 and psi2 must hold the same number of states")
    e1 = np.ascontiguousarray(eps1, dtype=np.float64)
    e2 = np.ascontiguousarray(eps2, dtype=np.float64)
    if e1.shape != (n,) or e2.shape != (n,):
        raise ValueError("one energy per state")
    out = torch.empty((n, ctxk.npw), dtype=torch.complex128, device=psi1.device) if states else None
    eps = np.zeros(n)
    dp = C.POINTER(C.c_double)
    _check(ctx1._lib.pw_kinterp(ctx1.handle, ctx2.handle, ctxk.handle, float(alpha), n, C.c_void_p(psi1.data_ptr()),
                                psi1.stride(0), e1.ctypes.data_as(dp), C.c_void_p(psi2.data_ptr()), psi2.stride(0),
                                e2.ctypes.data_as(dp), eps.ctypes.data_as(dp),
                                C.c_void_p(out.data_ptr() if out is not None else None),
                                out.stride(0) if out is not None else 0, _stream_ptr(stream)))
    return eps, out


def batch_solve(ctxs, e_refs, psis, opts=None, hist_len=0, stream=None, raise_on_noconv=True, **kw):
    """Folded-spectrum PCG of independent problems in one batched call (one
    context and one complex128 block [nb, npw_p] per problem, same nb).
    Returns (eigs, resids, stats, status): lists of per-problem arrays/dicts and
    the per-problem status codes."""
    n = len(ctxs)
    if not (n == len(e_refs) == len(psis)) or n == 0:
        raise ValueError("ctxs, e_refs and psis must have the same non-zero length")
    nb = psis[0].shape[0]
    for c, p in zip(ctxs, psis):
        _check_block(p, c.npw)
        if p.shape[0] != nb:
            raise ValueError("every block must have the same number of bands")
    o = opts if opts is not None else cg_opts(**kw)
    ctx_arr = (C.c_void_p * n)(*[c.handle for c in ctxs])
    e_arr = np.ascontiguousarray(e_refs, dtype=np.float64)
    psi_arr = (C.c_void_p * n)(*[p.data_ptr() for p in psis])
    ld_arr = np.array([p.stride(0) for p in psis], dtype=np.int64)
    eigs = [np.zeros(nb) for _ in range(n)]
    ress = [np.zeros(nb) for _ in range(n)]
    eig_arr = (C.c_void_p * n)(*[e.ctypes.data for e in eigs])
    res_arr = (C.c_void_p * n)(*[r.ctypes.data for r in ress])
    st_arr = (pw_cg_stats * n)()
    hists = [np.zeros((max(hist_len, 0), 2)) for _ in range(n)]
    for s_, h in zip(st_arr, hists):
        s_.n_hist = int(hist_len)
        s_.hist = h.ctypes.data_as(C.POINTER(C.c_double)) if hist_len else C.POINTER(C.c_double)()
    status = np.zeros(n, dtype=np.int32)
    rc = lib().pw_batch_solve(n, ctx_arr, e_arr.ctypes.data, nb, psi_arr, ld_arr.ctypes.data, eig_arr, res_arr,
                              C.byref(o), st_arr, status.ctypes.data, _stream_ptr(stream))
    stats = [dict(iters=s.iters, converged=bool(s.converged), n_hpsi=s.n_hpsi, max_resid=s.max_resid,
                  seconds=s.seconds, hist=h[:s.n_hist].copy(), fused=bool(s.fused), recoveries=s.recoveries)
             for s, h in zip(st_arr, hists)]
    if rc != PW_OK and not (rc == PW_ENOCONV and not raise_on_noconv):
        _check(rc)
    return eigs, ress, stats, status


FFT_PASSES = ("z_inverse", "xy_fft_v", "z_forward_kinetic")


def _cand_dict(c):
    return dict(pass_=c.pass_, kind=c.kind, nthr=c.nthr, sched=c.sched, radix=list(c.radix[:c.nradix]), ms=c.ms,
                chosen=bool(c.chosen))


def autotune(ctx, nb, dtype=PW_C128, reps=5, stream=None):
    """Time every FFT launch variant of this context's grid on nb bands, install the
    fastest per pass for `dtype`; returns the candidate records (dicts)."""
    cap = 256
    arr = (pw_fft_cand * cap)()
    n = C.c_int32(0)
    _check(lib().pw_ctx_autotune(ctx.handle, int(dtype), int(nb), int(reps), arr, cap, C.byref(n),
                                 _stream_ptr(stream)))
    return [_cand_dict(arr[i]) for i in range(min(n.value, cap))]


def fft_choose(ctx, cand, dtype=PW_C128):
    """Install one candidate (dict with pass_, kind, nthr, sched) for `dtype`."""
    c = pw_fft_cand()
    c.pass_, c.kind, c.nthr, c.sched = int(cand["pass_"]), int(cand["kind"]), int(cand.get("nthr", 0)), \
        int(cand.get("sched", 0))
    rad = list(cand.get("radix", []))[:12]
    c.nradix = len(rad)
    for i, v in enumerate(rad):
        c.radix[i] = int(v)
    _check(lib().pw_ctx_fft_choose(ctx.handle, int(dtype), C.byref(c)))
