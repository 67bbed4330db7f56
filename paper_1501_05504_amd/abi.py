"""Thin ctypes binding of libdmrg3s (include/dmrg3s.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Tensors are torch tensors on the GPU (device memory and streams are
all torch is used for); their data pointers and the current HIP stream are
handed to the C-ABI.  Importing this module loads the library and raises
ImportError when it has not been built.
"""
import ctypes
import weakref
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdmrg3s.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libdmrg3s.so is not built (run __graft_entry__.build() or "
                      "python paper_1501_05504_amd/build_lib.py): " + LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

F64, F32, BF16 = 0, 1, 2
L2R, R2L = 0, 1
OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, ENUMERIC = 0, 1, -1, -2, -3, -4
_PREC = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}

c_int, c_long, c_double, c_void_p = ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_void_p
c_int_p, c_double_p = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)


_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p, c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


class d3s_allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", c_void_p)]


def torch_allocator(device):
    """(alloc, free) callbacks that take the library's device memory (its
    workspace and the tables of block plans) from torch's caching allocator,
    stream-ordered on the stream the library passes; a failed allocation
    returns NULL, which the library reports as D3S_ENOMEM."""
    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except Exception:
            return None

    def free(ptr, stream, user):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


class d3s_state(ctypes.Structure):
    _fields_ = [("l", c_int), ("d", c_int), ("mmax", c_int), ("m", c_int_p), ("w", c_int_p),
                ("site", ctypes.POINTER(c_void_p)), ("mpo", ctypes.POINTER(c_void_p)),
                ("lenv", ctypes.POINTER(c_void_p)), ("renv", ctypes.POINTER(c_void_p)),
                ("center", c_int)]


class d3s_sweep_params(ctypes.Structure):
    _fields_ = [("alpha", c_double), ("adaptive_alpha", c_int), ("eps", c_double),
                ("lanczos_tol", c_double), ("lanczos_kmax", c_int), ("lanczos_max_matvecs", c_int),
                ("prec", c_int), ("e_before", c_double), ("m_limit", c_int), ("mixed_min_gflop", c_double),
                ("expansion", c_int)]


class d3s_site_record(ctypes.Structure):
    _fields_ = [("site", c_int), ("dir", c_int), ("k", c_int), ("matvecs", c_int), ("f64_matvecs", c_int),
                ("e_before", c_double), ("lam", c_double), ("e_f", c_double), ("alpha", c_double),
                ("discarded", c_double), ("t_eig", c_double), ("t_expand", c_double),
                ("t_trunc", c_double), ("t_env", c_double), ("t_energy", c_double),
                ("t_trunc_eig", c_double), ("trunc_passes", c_int), ("reserved_", c_int)]


class d3s_sweep_stats(ctypes.Structure):
    _fields_ = [("capacity", c_int), ("count", c_int), ("records", ctypes.POINTER(d3s_site_record)),
                ("energy", c_double), ("seconds", c_double), ("nonconverged", c_int)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_create = _sig("d3s_create", c_int, [ctypes.POINTER(c_void_p), c_int, c_void_p, ctypes.POINTER(d3s_allocator)])
_destroy = _sig("d3s_destroy", None, [c_void_p])
_last_error = _sig("d3s_last_error", ctypes.c_char_p, [c_void_p])
_set_stream = _sig("d3s_set_stream", c_int, [c_void_p, c_void_p])
_synchronize = _sig("d3s_synchronize", c_int, [c_void_p])
_version = _sig("d3s_version", ctypes.c_char_p, [])
_set_tile_config = _sig("d3s_set_tile_config", c_int, [c_void_p, c_int])
_set_splitk = _sig("d3s_set_splitk", c_int, [c_void_p, c_int])
_set_gtile = _sig("d3s_set_grouped_tile", c_int, [c_void_p, c_int])
_set_bsplit = _sig("d3s_set_block_split", c_int, [c_void_p, c_double])
_set_autotune = _sig("d3s_set_autotune", c_int, [c_void_p, c_int, ctypes.c_char_p])
_set_eig = _sig("d3s_set_eigensolver", c_int, [c_void_p, c_int, c_int])
_eig_batched = _sig("d3s_eig_batched", c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p])
_tridiag = _sig("d3s_tridiag_lowest", c_int, [c_int, c_double_p, c_double_p, c_double_p, c_double_p])
_profile_begin = _sig("d3s_profile_begin", c_int, [c_void_p, c_int])
_profile_end = _sig("d3s_profile_end", c_int, [c_void_p, c_double_p, c_int_p])
_apply_heff = _sig("d3s_apply_heff", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 5)
_apply_heff2 = _sig("d3s_apply_heff_two_site", c_int, [c_void_p, c_int] + [c_int] * 6 + [c_void_p] * 6)
_cwf_env = _sig("d3s_cwf_environment", c_int, [c_void_p] + [c_int] * 4 + [c_void_p] * 3)
_apply_cwf = _sig("d3s_apply_cwf", c_int, [c_void_p, c_int] + [c_int] * 3 + [c_void_p] * 4)
_apply_heff_noalloc = _sig("d3s_apply_heff_noalloc", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 5)
_expand = _sig("d3s_expand_subspace", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 3 +
               [c_double, c_void_p])
_truncate = _sig("d3s_truncate", c_int, [c_void_p, c_int, c_int, c_int, c_int, c_long, c_void_p, c_void_p,
                                         c_int, c_double, c_void_p, c_long, c_void_p, c_void_p, c_int,
                                         c_double_p, c_int_p, c_double_p])
_update_env = _sig("d3s_update_env", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 4)
_update_env_h2 = _sig("d3s_update_env_h2", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 4)
_residual_gram = _sig("d3s_residual_gram", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 5 +
                      [c_double, c_double, c_void_p])
_residual_expand = _sig("d3s_residual_expand", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 5 +
                        [c_double, c_double, c_void_p, ctypes.POINTER(c_long)])
_lanczos = _sig("d3s_lanczos", c_int, [c_void_p, c_int] + [c_int] * 5 + [c_void_p] * 4 +
                [c_double, c_int, c_int, c_double_p, c_int_p])
_energy = _sig("d3s_energy", c_int, [c_void_p] + [c_int] * 5 + [c_void_p] * 4 + [c_double_p])
_grad_w = _sig("d3s_heff_grad_W", c_int, [c_void_p] + [c_int] * 5 + [c_void_p] * 5)
_prepare = _sig("d3s_prepare", c_int, [c_void_p, ctypes.POINTER(d3s_state), c_double_p])
_sweep = _sig("d3s_sweep", c_int, [c_void_p, ctypes.POINTER(d3s_state), ctypes.POINTER(d3s_sweep_params),
                                   ctypes.POINTER(d3s_sweep_stats)])
_grads = _sig("d3s_energy_gradients", c_int, [c_void_p, ctypes.POINTER(d3s_state), ctypes.POINTER(c_void_p)])
_mpo_spin = _sig("d3s_mpo_spin_exchange", c_int, [c_int, c_int, c_double_p, c_double_p,
                                                  ctypes.POINTER(c_long), c_int_p, ctypes.POINTER(c_long)])
_mpo_fermion = _sig("d3s_mpo_fermion_hopping", c_int, [c_int, c_int, c_double_p, c_double, c_double_p,
                                                       c_double_p, ctypes.POINTER(c_long), c_int_p,
                                                       ctypes.POINTER(c_long)])


class d3s_sectors(ctypes.Structure):
    _fields_ = [("nsec", c_int), ("q", c_int_p), ("dim", c_int_p)]


_plan_create = _sig("d3s_block_plan_create", c_int, [c_void_p, c_int, c_int, c_int, c_int,
                                                     ctypes.POINTER(d3s_sectors), ctypes.POINTER(d3s_sectors),
                                                     c_int_p, c_int_p, c_int_p, ctypes.POINTER(c_void_p),
                                                     c_double_p, c_int_p])
_set_eig_workers = _sig("d3s_set_eig_workers", c_int, [c_void_p, c_int])
_set_refine = _sig("d3s_set_refinement", c_int, [c_void_p, c_double, c_int, c_double])
_plan_create_layout = _sig("d3s_block_plan_create_layout", c_int,
                           [c_void_p, c_int, c_int, c_int, c_int, ctypes.POINTER(d3s_sectors),
                            ctypes.POINTER(d3s_sectors), c_int_p, c_int_p, c_int_p, c_int,
                            ctypes.POINTER(c_void_p), c_double_p, c_int_p])
_plan_sizes = _sig("d3s_block_plan_sizes", c_int, [c_void_p, ctypes.POINTER(c_long), ctypes.POINTER(c_long),
                                                   ctypes.POINTER(c_long)])
_plan_bind = _sig("d3s_block_plan_bind", c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p])
_apply_bound = _sig("d3s_apply_heff_blocks_bound", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int])
_plan_destroy = _sig("d3s_block_plan_destroy", None, [c_void_p, c_void_p])
_apply_blocks = _sig("d3s_apply_heff_blocks", c_int, [c_void_p, c_void_p, c_int] + [c_void_p] * 5 + [c_int])
_expand_blocks = _sig("d3s_expand_subspace_blocks", c_int,
                      [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_double, c_void_p])
_trunc_blocks = _sig("d3s_truncate_blocks", c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_int, c_double,
                                                    c_void_p, c_long, c_void_p, c_void_p, c_int, c_int, c_int_p,
                                                    c_int_p, c_int_p, c_int_p, c_double_p])
_env_blocks = _sig("d3s_update_env_blocks", c_int, [c_void_p, c_void_p, c_int] + [c_void_p] * 4)
_spin_charges = _sig("d3s_mpo_spin_charges", c_int, [c_int, c_int_p])
_fermion_charges = _sig("d3s_mpo_fermion_charges", c_int, [c_int, c_int_p])


class d3s_symmetry(ctypes.Structure):
    _fields_ = [("nq", c_int), ("phys_q", c_int_p), ("mpo_q", ctypes.POINTER(c_int_p)), ("maxsec", c_int),
                ("nsec", c_int_p), ("sec_q", ctypes.POINTER(c_int_p)), ("sec_dim", ctypes.POINTER(c_int_p)),
                ("env_cap", ctypes.c_long)]


_prepare_blocks = _sig("d3s_prepare_blocks", c_int, [c_void_p, ctypes.POINTER(d3s_state),
                                                     ctypes.POINTER(d3s_symmetry), c_double_p])
_sweep_blocks = _sig("d3s_sweep_blocks", c_int, [c_void_p, ctypes.POINTER(d3s_state), ctypes.POINTER(d3s_symmetry),
                                                 ctypes.POINTER(d3s_sweep_params), ctypes.POINTER(d3s_sweep_stats),
                                                 c_int])


class D3SError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("dmrg3s status %d: %s" % (status, msg))
        self.status = status


def version():
    return _version().decode()


def tridiag_lowest(alpha, beta):
    """Lowest eigenpair of a symmetric tridiagonal matrix (host helper of the
    eigensolver): returns (theta, y) as (float, numpy array)."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if b.size != max(a.size - 1, 0):
        raise ValueError("beta must have len(alpha) - 1 entries")
    y = np.empty_like(a)
    th = c_double()
    st = _tridiag(a.size, a.ctypes.data_as(c_double_p), b.ctypes.data_as(c_double_p) if b.size else None,
                  ctypes.byref(th), y.ctypes.data_as(c_double_p))
    if st != OK:
        raise D3SError(st, "d3s_tridiag_lowest")
    return th.value, y


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n, dtype, name):
    """A kernel reads or writes n elements of t: refuse anything smaller, on
    the host, before the call."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < n:
        raise ValueError("%s holds %d elements, the call needs %d" % (name, t.numel(), n))


_ELT = {F64: (torch.float64, torch.float64, torch.float64),     # (L/R/psi, W, out)
        F32: (torch.float32, torch.float32, torch.float32),
        BF16: (torch.bfloat16, torch.float32, torch.float32)}


class Context:
    """A library context bound to a device and to torch's current stream.
    allocator: "torch" (default: torch's caching allocator owns every device
    buffer of the library), None (the library's hipMalloc), or a pair of
    Python callables alloc(nbytes, stream, user) -> address or None and
    free(address, stream, user)."""

    def __init__(self, device=0, allocator="torch"):
        self.device = device
        h = c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        self._alloc = None
        if allocator is not None:
            fa, ff = torch_allocator(device) if allocator == "torch" else allocator
            # the callbacks must outlive the context
            self._alloc = d3s_allocator(_ALLOC_FN(fa), _FREE_FN(ff), None)
        st = _create(ctypes.byref(h), device, c_void_p(stream),
                     ctypes.byref(self._alloc) if self._alloc is not None else None)
        if st != OK:
            raise D3SError(st, "d3s_create failed")
        self.h = h
        self._plans = weakref.WeakSet()      # block plans whose tables this context holds

    def close(self):
        if self.h:
            for p in list(self._plans):
                p.close()
            _destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, warn_ok=False):
        if st == OK or (warn_ok and st == ENOCONV):
            return st
        raise D3SError(st, _last_error(self.h).decode())

    def _sync_stream(self):
        self._check(_set_stream(self.h, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    def synchronize(self):
        self._check(_synchronize(self.h))

    def set_tile_config(self, cfg):
        """-1 size rule (default); 0: 128x128 (4 waves), 1: 64x64, 2: 256x128
        (8 waves), 3: 128x128 (8 waves), 4: 256x128 (4 waves; FP32/BF16)."""
        self._check(_set_tile_config(self.h, int(cfg)))

    def set_autotune(self, enable, cache_path=None):
        self._check(_set_autotune(self.h, 1 if enable else 0,
                                  None if cache_path is None else str(cache_path).encode()))

    def eig_batched(self, A, W):
        """A: (batch, n, n) FP64 device tensor of symmetric matrices (the
        eigensolver reads them column-major, i.e. A[b].T); replaced by the
        eigenvectors (row j of A[b] = eigenvector j); W: (batch, n) receives
        the eigenvalues, ascending."""
        self._sync_stream()
        if A.dim() != 3 or A.shape[1] != A.shape[2]:
            raise ValueError("A must be (batch, n, n)")
        batch, n = A.shape[0], A.shape[1]
        _need(A, batch * n * n, torch.float64, "A")
        _need(W, batch * n, torch.float64, "W")
        return self._check(_eig_batched(self.h, n, batch, _ptr(A), _ptr(W)))

    def set_eigensolver(self, kind, jacobi_max_n=0):
        """0 auto (Jacobi up to jacobi_max_n), 1 divide and conquer, 2 Jacobi,
        3 the library's LDS solver up to n = 128."""
        self._check(_set_eig(self.h, int(kind), int(jacobi_max_n)))

    def set_eig_workers(self, workers):
        """Concurrent divide-and-conquer solves in a truncation (1 = one at a time)."""
        self._check(_set_eig_workers(self.h, int(workers)))

    def set_refinement(self, eta=0.1, inner_max=20, low_tol=0.0):
        """Mixed-precision eigensolver: inner CG target eta (relative to the
        FP64 residual), its step cap, and the low-precision Lanczos stop
        (<= 0: the per-precision default)."""
        self._check(_set_refine(self.h, float(eta), int(inner_max), float(low_tol)))

    def set_block_split(self, min_gflop):
        """Split the block sweeps' second GEMM from min_gflop GFLOP on (< 0: never)."""
        self._check(_set_bsplit(self.h, float(min_gflop)))

    def set_grouped_tile(self, cfg):
        """-1 rule/autotuner; 0: 128x128, 1: 64x64, 2: 96x96, 3: 32x32 (4 waves),
        4: 128x128, 5: 256x128 (8 waves)."""
        self._check(_set_gtile(self.h, int(cfg)))

    def set_splitk(self, enable):
        self._check(_set_splitk(self.h, 1 if enable else 0))

    def profile_begin(self, capacity):
        self._check(_profile_begin(self.h, capacity))

    def profile_end(self):
        """Returns ([ms GEMM-1, ms W-map, ms GEMM-2] summed, number of calls)."""
        ms = (ctypes.c_double * 3)()
        n = c_int()
        self._check(_profile_end(self.h, ms, ctypes.byref(n)))
        return list(ms), n.value

    # --- the hot path ---------------------------------------------------
    def apply_heff(self, L, W, R, psi, out):
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        prec = _PREC[psi.dtype]
        te, tw, to = _ELT[prec]
        _need(L, ml * wl * ml, te, "L")
        _need(W, wl * wr * d * d, tw, "W")
        _need(R, mr * wr * mr, te, "R")
        _need(psi, ml * d * mr, te, "psi")
        _need(out, ml * d * mr, to, "out")
        return self._check(_apply_heff(self.h, prec, ml, d, mr, wl, wr, _ptr(L), _ptr(W), _ptr(R),
                                       _ptr(psi), _ptr(out)))

    def apply_heff_noalloc(self, L, W, R, psi, out):
        """apply_heff whose intermediates live in the library's fixed 64 MiB
        per-GPU scratch array (no device allocation)."""
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        prec = _PREC[psi.dtype]
        te, tw, to = _ELT[prec]
        _need(L, ml * wl * ml, te, "L")
        _need(W, wl * wr * d * d, tw, "W")
        _need(R, mr * wr * mr, te, "R")
        _need(psi, ml * d * mr, te, "psi")
        _need(out, ml * d * mr, to, "out")
        return self._check(_apply_heff_noalloc(self.h, prec, ml, d, mr, wl, wr, _ptr(L), _ptr(W), _ptr(R),
                                               _ptr(psi), _ptr(out)))

    def apply_heff_two_site(self, L, W1, W2, R, psi2, out):
        """Two-site H_eff * psi2, psi2 and out (ml, d, d, mr); FP64 or FP32."""
        self._sync_stream()
        ml, d, d2, mr = psi2.shape
        wl, wc, wr = W1.shape[0], W1.shape[1], W2.shape[1]
        if d2 != d or W2.shape[0] != wc:
            raise ValueError("two-site shapes do not match")
        prec = _PREC[psi2.dtype]
        if prec == BF16:
            raise ValueError("two-site H_eff takes float64 or float32")
        t = psi2.dtype
        _need(L, ml * wl * ml, t, "L")
        _need(W1, wl * wc * d * d, t, "W1")
        _need(W2, wc * wr * d * d, t, "W2")
        _need(R, mr * wr * mr, t, "R")
        _need(psi2, ml * d * d * mr, t, "psi2")
        _need(out, ml * d * d * mr, t, "out")
        return self._check(_apply_heff2(self.h, prec, ml, d, mr, wl, wc, wr, _ptr(L), _ptr(W1), _ptr(W2),
                                        _ptr(R), _ptr(psi2), _ptr(out)))

    def cwf_environment(self, L, W, Lt):
        """Lt[(a,s), v, (x,t)] = sum_w L[a,w,x] W[w,v,s,t], FP64."""
        self._sync_stream()
        ml, wl = L.shape[0], L.shape[1]
        wr, d = W.shape[1], W.shape[2]
        f = torch.float64
        _need(L, ml * wl * ml, f, "L")
        _need(W, wl * wr * d * d, f, "W")
        _need(Lt, ml * d * wr * ml * d, f, "Lt")
        return self._check(_cwf_env(self.h, ml, d, wl, wr, _ptr(L), _ptr(W), _ptr(Lt)))

    def apply_cwf(self, Lt, R, C, out):
        """out[(a,s), b] = sum Lt[(a,s),v,(x,t)] C[(x,t),y] R[b,v,y]; FP64 or FP32."""
        self._sync_stream()
        mlp, mr = C.shape
        wr = R.shape[1]
        prec = _PREC[C.dtype]
        if prec == BF16:
            raise ValueError("the centre-matrix application takes float64 or float32")
        t = C.dtype
        _need(Lt, mlp * wr * mlp, t, "Lt")
        _need(R, mr * wr * mr, t, "R")
        _need(C, mlp * mr, t, "C")
        _need(out, mlp * mr, t, "out")
        return self._check(_apply_cwf(self.h, prec, mlp, mr, wr, _ptr(Lt), _ptr(R), _ptr(C), _ptr(out)))

    def expand_subspace(self, direction, env, W, psi, alpha, Mtilde):
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        f = torch.float64
        _need(W, wl * wr * d * d, f, "W")
        _need(psi, ml * d * mr, f, "psi")
        if direction == L2R:
            _need(env, ml * wl * ml, f, "L")
            _need(Mtilde, ml * d * (1 + wr) * mr, f, "Mtilde")
        else:
            _need(env, mr * wr * mr, f, "R")
            _need(Mtilde, (1 + wl) * ml * d * mr, f, "Mtilde")
        return self._check(_expand(self.h, direction, ml, d, mr, wl, wr, _ptr(env), _ptr(W), _ptr(psi),
                                   float(alpha), _ptr(Mtilde)))

    def truncate(self, direction, Mtilde, psi, kmax, rel_cutoff, nbr, site_out, nbr_out, renormalize=True):
        """Returns (k, discarded, singular values).  nbr=None: nbr_out receives
        S_k V_k^T (L2R) or U_k S_k (R2L), the split of a two-site tensor."""
        self._sync_stream()
        ml, d, mr = psi.shape
        f = torch.float64
        if direction == L2R:
            width = Mtilde.shape[1]
            other = nbr.numel() // mr if nbr is not None else mr
            n = ml * d
            if Mtilde.shape[0] != n:
                raise ValueError("L2R: Mtilde must have m_l*d rows")
            if nbr is not None:
                _need(nbr, mr * other, f, "nbr")
            _need(site_out, n * min(kmax, n), f, "site_out")
            _need(nbr_out, min(kmax, n) * other, f, "nbr_out")
        else:
            width = Mtilde.shape[0]
            other = nbr.numel() // ml if nbr is not None else ml
            n = d * mr
            if Mtilde.shape[1] != n:
                raise ValueError("R2L: Mtilde must have d*m_r columns")
            if nbr is not None:
                _need(nbr, ml * other, f, "nbr")
            _need(site_out, n * min(kmax, n), f, "site_out")
            _need(nbr_out, min(kmax, n) * other, f, "nbr_out")
        _need(Mtilde, Mtilde.shape[0] * Mtilde.shape[1], f, "Mtilde")
        _need(psi, ml * d * mr, f, "psi")
        s = (ctypes.c_double * n)()
        k = c_int()
        disc = c_double()
        self._check(_truncate(self.h, direction, ml, d, mr, width, _ptr(Mtilde), _ptr(psi), kmax,
                              float(rel_cutoff), _ptr(nbr) if nbr is not None else None, other,
                              _ptr(site_out), _ptr(nbr_out),
                              1 if renormalize else 0, s, ctypes.byref(k), ctypes.byref(disc)))
        return k.value, disc.value, list(s)

    def update_env_h2(self, direction, env_in, W, site, env_out):
        """Environment of the channel pairs of H^2: L2R env_in (ml, wl^2, ml) ->
        env_out (mr, wr^2, mr); R2L env_in (mr, wr^2, mr) -> env_out (ml, wl^2, ml)."""
        self._sync_stream()
        ml, d, mr = site.shape
        wl, wr = W.shape[0], W.shape[1]
        f = torch.float64
        _need(W, wl * wr * d * d, f, "W")
        _need(site, ml * d * mr, f, "site")
        if direction == L2R:
            _need(env_in, ml * wl * wl * ml, f, "env_in")
            _need(env_out, mr * wr * wr * mr, f, "env_out")
        else:
            _need(env_in, mr * wr * wr * mr, f, "env_in")
            _need(env_out, ml * wl * wl * ml, f, "env_out")
        return self._check(_update_env_h2(self.h, direction, ml, d, mr, wl, wr, _ptr(env_in), _ptr(W),
                                          _ptr(site), _ptr(env_out)))

    def residual_gram(self, direction, L, R, h2, W, psi, energy, alpha, gram):
        """Gram matrix of the expanded tensor with the exact residual as its
        expansion part: (ml d)^2 for L2R (h2 = right H^2 environment), (d mr)^2
        for R2L (h2 = left one)."""
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        f = torch.float64
        _need(L, ml * wl * ml, f, "L")
        _need(R, mr * wr * mr, f, "R")
        _need(W, wl * wr * d * d, f, "W")
        _need(psi, ml * d * mr, f, "psi")
        if direction == L2R:
            _need(h2, mr * wr * wr * mr, f, "h2")
            _need(gram, (ml * d) ** 2, f, "gram")
        else:
            _need(h2, ml * wl * wl * ml, f, "h2")
            _need(gram, (d * mr) ** 2, f, "gram")
        return self._check(_residual_gram(self.h, direction, ml, d, mr, wl, wr, _ptr(L), _ptr(R), _ptr(h2),
                                          _ptr(W), _ptr(psi), float(energy), float(alpha), _ptr(gram)))

    def residual_expand(self, direction, L, R, h2, W, psi, energy, alpha, Mt):
        """The exact-residual expanded tensor on an orthonormal basis of its
        far-side vectors, written into Mt (capacity (ml d)(2+wr) mr for L2R,
        (2+wl) ml (d mr) for R2L); returns its row length (L2R, mr + r) or row
        count (R2L, ml + r).  Pass the matrix it fills to truncate()."""
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        f = torch.float64
        _need(L, ml * wl * ml, f, "L")
        _need(R, mr * wr * mr, f, "R")
        _need(W, wl * wr * d * d, f, "W")
        _need(psi, ml * d * mr, f, "psi")
        if direction == L2R:
            _need(h2, mr * wr * wr * mr, f, "h2")
            _need(Mt, ml * d * (2 + wr) * mr, f, "Mt")
        else:
            _need(h2, ml * wl * wl * ml, f, "h2")
            _need(Mt, (2 + wl) * ml * d * mr, f, "Mt")
        ext = c_long()
        self._check(_residual_expand(self.h, direction, ml, d, mr, wl, wr, _ptr(L), _ptr(R), _ptr(h2), _ptr(W),
                                     _ptr(psi), float(energy), float(alpha), _ptr(Mt), ctypes.byref(ext)))
        return ext.value

    def update_env(self, direction, env_in, W, site, env_out):
        self._sync_stream()
        ml, d, mr = site.shape
        wl, wr = W.shape[0], W.shape[1]
        f = torch.float64
        _need(W, wl * wr * d * d, f, "W")
        _need(site, ml * d * mr, f, "site")
        if direction == L2R:
            _need(env_in, ml * wl * ml, f, "L")
            _need(env_out, mr * wr * mr, f, "env_out")
        else:
            _need(env_in, mr * wr * mr, f, "R")
            _need(env_out, ml * wl * ml, f, "env_out")
        return self._check(_update_env(self.h, direction, ml, d, mr, wl, wr, _ptr(env_in), _ptr(W),
                                       _ptr(site), _ptr(env_out)))

    def lanczos(self, L, W, R, psi, tol=1e-12, kmax=40, max_matvecs=2000, prec=F64):
        """Returns (theta, matvecs, converged); psi is overwritten by the Ritz vector."""
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        self._check_heff_f64(L, W, R, psi, ml, d, mr, wl, wr)
        th = c_double()
        nmv = c_int()
        st = self._check(_lanczos(self.h, prec, ml, d, mr, wl, wr, _ptr(L), _ptr(W), _ptr(R), _ptr(psi),
                                  float(tol), kmax, max_matvecs, ctypes.byref(th), ctypes.byref(nmv)),
                         warn_ok=True)
        return th.value, nmv.value, st == OK

    def _check_heff_f64(self, L, W, R, psi, ml, d, mr, wl, wr):
        f = torch.float64
        _need(L, ml * wl * ml, f, "L")
        _need(W, wl * wr * d * d, f, "W")
        _need(R, mr * wr * mr, f, "R")
        _need(psi, ml * d * mr, f, "psi")

    def energy(self, L, W, R, psi):
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = W.shape[0], W.shape[1]
        self._check_heff_f64(L, W, R, psi, ml, d, mr, wl, wr)
        e = c_double()
        self._check(_energy(self.h, ml, d, mr, wl, wr, _ptr(L), _ptr(W), _ptr(R), _ptr(psi),
                            ctypes.byref(e)))
        return e.value

    def heff_grad_W(self, L, R, psi, ybar, Wbar):
        self._sync_stream()
        ml, d, mr = psi.shape
        wl, wr = Wbar.shape[0], Wbar.shape[1]
        self._check_heff_f64(L, Wbar, R, psi, ml, d, mr, wl, wr)
        _need(ybar, ml * d * mr, torch.float64, "ybar")
        return self._check(_grad_w(self.h, ml, d, mr, wl, wr, _ptr(L), _ptr(R), _ptr(psi), _ptr(ybar),
                                   _ptr(Wbar)))

    def prepare(self, state):
        self._sync_stream()
        e = c_double()
        self._check(_prepare(self.h, ctypes.byref(state.c), ctypes.byref(e)))
        state.pull_dims()
        return e.value

    def energy_gradients(self, state):
        """dE/dW_i for every site (list of device tensors shaped like the MPO)."""
        self._sync_stream()
        grads = [torch.empty_like(w) for w in state.mpo]
        arr = (c_void_p * state.l)(*[g.data_ptr() for g in grads])
        self._check(_grads(self.h, ctypes.byref(state.c), arr))
        state.pull_dims()
        return grads

    def prepare_blocks(self, state, sym):
        self._sync_stream()
        e = c_double()
        sym.c.env_cap = state.env_cap
        self._check(_prepare_blocks(self.h, ctypes.byref(state.c), ctypes.byref(sym.c), ctypes.byref(e)))
        state.pull_dims()
        return e.value

    def sweep_blocks(self, state, sym, params, use_graph=True):
        self._sync_stream()
        cap = 2 * state.l
        recs = (d3s_site_record * cap)()
        stats = d3s_sweep_stats(cap, 0, recs, 0.0, 0.0, 0)
        sym.c.env_cap = state.env_cap
        st = self._check(_sweep_blocks(self.h, ctypes.byref(state.c), ctypes.byref(sym.c), ctypes.byref(params),
                                       ctypes.byref(stats), 1 if use_graph else 0), warn_ok=True)
        state.pull_dims()
        return st, stats, [recs[i] for i in range(min(stats.count, cap))]

    def sweep(self, state, params):
        """One full sweep; returns (status, stats, records)."""
        self._sync_stream()
        cap = 2 * state.l
        recs = (d3s_site_record * cap)()
        stats = d3s_sweep_stats(cap, 0, recs, 0.0, 0.0, 0)
        st = self._check(_sweep(self.h, ctypes.byref(state.c), ctypes.byref(params), ctypes.byref(stats)),
                         warn_ok=True)
        state.pull_dims()
        return st, stats, [recs[i] for i in range(min(stats.count, cap))]


class State:
    """Device buffers of an MPS, its MPO and its environments (torch-owned),
    described to the library by a d3s_state."""

    def __init__(self, mpo_blocks, site_tensors, mmax, device="cuda", env_cap=None):
        """env_cap: elements per environment buffer (default the dense size
        mmax*wmax*mmax).  The block-sparse calls store environments packed
        and can run with far smaller buffers; the dense calls need the
        default."""
        self.l = len(site_tensors)
        self.d = site_tensors[0].shape[1]
        self.mmax = mmax
        w = [1] + [int(b.shape[1]) for b in mpo_blocks]
        self.wmax = max(w)
        cap_site = mmax * self.d * mmax
        cap_env = mmax * self.wmax * mmax if env_cap is None else int(env_cap)
        self.env_cap = cap_env
        self.site = [torch.zeros(cap_site, dtype=torch.float64, device=device) for _ in range(self.l)]
        self.lenv = [torch.zeros(cap_env, dtype=torch.float64, device=device) for _ in range(self.l)]
        self.renv = [torch.zeros(cap_env, dtype=torch.float64, device=device) for _ in range(self.l)]
        self.mpo = [torch.as_tensor(b, dtype=torch.float64).contiguous().to(device) for b in mpo_blocks]
        m = [1] + [int(t.shape[2]) for t in site_tensors]
        if len(mpo_blocks) != self.l:
            raise ValueError("one MPO tensor per site is required")
        for i, t in enumerate(site_tensors):
            if tuple(t.shape) != (m[i], self.d, m[i + 1]) or m[i + 1] > mmax or m[i] > mmax:
                raise ValueError("site %d has shape %s, expected (%d, %d, %d) with bonds <= %d"
                                 % (i, tuple(t.shape), m[i], self.d, m[i + 1], mmax))
            if tuple(mpo_blocks[i].shape) != (w[i], w[i + 1], self.d, self.d):
                raise ValueError("MPO tensor %d has shape %s" % (i, tuple(mpo_blocks[i].shape)))
        if m[-1] != 1 or w[-1] != 1 or mpo_blocks[0].shape[0] != 1:
            raise ValueError("open boundaries need m_l = w_l = 1 at both ends")
        for i, t in enumerate(site_tensors):
            tt = torch.as_tensor(t, dtype=torch.float64).reshape(-1)
            self.site[i][: tt.numel()].copy_(tt.to(device))
        self._m = (c_int * (self.l + 1))(*m)
        self._w = (c_int * (self.l + 1))(*w)
        self._site = (c_void_p * self.l)(*[t.data_ptr() for t in self.site])
        self._mpo = (c_void_p * self.l)(*[t.data_ptr() for t in self.mpo])
        self._lenv = (c_void_p * self.l)(*[t.data_ptr() for t in self.lenv])
        self._renv = (c_void_p * self.l)(*[t.data_ptr() for t in self.renv])
        self.c = d3s_state(self.l, self.d, mmax, self._m, self._w, self._site, self._mpo, self._lenv,
                           self._renv, self.l - 1)
        self.m = list(m)
        self.w = list(w)

    def pull_dims(self):
        self.m = [self._m[i] for i in range(self.l + 1)]

    def site_tensor(self, i):
        n = self.m[i] * self.d * self.m[i + 1]
        return self.site[i][:n].reshape(self.m[i], self.d, self.m[i + 1])

    def tensors(self):
        return [self.site_tensor(i) for i in range(self.l)]


def save_checkpoint(path, state, sym=None, **scalars):
    """Checkpoint of a sweep (host side, an .npz file with arrays only): the
    site tensors of `state` (anything with .l and .tensors()), the sectors of
    every bond when `sym` is given (anything with .sectors(b)), and scalar
    values by keyword (for instance alpha, energy).  A sweep resumes from it
    through load_checkpoint: a State and a Symmetry rebuilt from the arrays,
    environments from prepare / prepare_blocks, and the saved alpha."""
    import numpy as np
    arrs = {"l": np.int64(state.l)}
    for i, t in enumerate(state.tensors()):
        arrs["site_%d" % i] = torch.as_tensor(t).detach().to("cpu", torch.float64).numpy()
    if sym is not None:
        for b in range(state.l + 1):
            q, d = sym.sectors(b)
            arrs["secq_%d" % b] = np.asarray(q, dtype=np.int32)
            arrs["secd_%d" % b] = np.asarray(d, dtype=np.int32)
    for k, v in scalars.items():
        arrs["scalar_" + k] = np.float64(v)
    with open(path, "wb") as f:
        np.savez(f, **arrs)


def load_checkpoint(path):
    """Inverse of save_checkpoint: {"tensors": [CPU FP64 tensors],
    "sectors": [(charges, dims) per bond] or None, and the scalars}.  Reads
    arrays only (no pickled objects)."""
    import numpy as np
    with np.load(path, allow_pickle=False) as z:
        l = int(z["l"])
        out = {"tensors": [torch.from_numpy(z["site_%d" % i].copy()) for i in range(l)],
               "sectors": ([(z["secq_%d" % b].copy(), z["secd_%d" % b].copy()) for b in range(l + 1)]
                           if "secq_0" in z.files else None)}
        for k in z.files:
            if k.startswith("scalar_"):
                out[k[len("scalar_"):]] = float(z[k])
    return out


class Symmetry:
    """Charges of a symmetric chain (d3s_symmetry): physical charges, MPO
    channel charges per MPO bond and the current sectors of every MPS bond."""

    def __init__(self, phys_q, mpo_channel_q, sectors, maxsec=4096):
        import numpy as np
        phys = np.ascontiguousarray(np.asarray(phys_q, dtype=np.int32))
        self.nq = phys.shape[1]
        self.l = len(sectors) - 1
        self.maxsec = maxsec
        self._phys = phys
        self._mpo = [np.ascontiguousarray(np.asarray(q, dtype=np.int32).reshape(-1, self.nq))
                     for q in mpo_channel_q]
        self._secq = [np.zeros(maxsec * self.nq, dtype=np.int32) for _ in sectors]
        self._secd = [np.zeros(maxsec, dtype=np.int32) for _ in sectors]
        self._nsec = (c_int * (self.l + 1))()
        for b, (q, dm) in enumerate(sectors):
            q = np.asarray(q, dtype=np.int32).reshape(-1, self.nq)
            n = len(dm)
            if n > maxsec:
                raise ValueError("more sectors than maxsec")
            self._secq[b][: n * self.nq] = q.ravel()
            self._secd[b][:n] = dm
            self._nsec[b] = n
        self._mpo_p = (c_int_p * (self.l + 1))(*[a.ctypes.data_as(c_int_p) for a in self._mpo])
        self._secq_p = (c_int_p * (self.l + 1))(*[a.ctypes.data_as(c_int_p) for a in self._secq])
        self._secd_p = (c_int_p * (self.l + 1))(*[a.ctypes.data_as(c_int_p) for a in self._secd])
        self.c = d3s_symmetry(self.nq, self._phys.ctypes.data_as(c_int_p), self._mpo_p, maxsec, self._nsec,
                              self._secq_p, self._secd_p, 0)

    def sectors(self, b):
        n = self._nsec[b]
        return self._secq[b][: n * self.nq].reshape(n, self.nq).copy(), self._secd[b][:n].copy()


def mpo_bond_charges(mpo_blocks, channel_q):
    """Channel charges of every MPO bond of a chain built by the builders
    above: the bulk bonds carry `channel_q`; the boundary bonds have one
    channel of charge 0."""
    import numpy as np
    nq = np.asarray(channel_q).shape[1]
    l = len(mpo_blocks)
    out = [np.zeros((1, nq), dtype=np.int32)]
    for i in range(1, l):
        out.append(np.asarray(channel_q, dtype=np.int32))
    out.append(np.zeros((1, nq), dtype=np.int32))
    return out


def sweep_params(alpha=1e-3, adaptive=True, eps=1e-14, tol=1e-12, kmax=40, max_matvecs=2000, prec=F64,
                 e_before=0.0, m_limit=0, mixed_min_gflop=2.0, expansion="heuristic"):
    """expansion: "heuristic" (the term P of eq. subexp-ourt) or "residual"
    (the exact residual H Psi - E Psi; dense sweeps only)."""
    if expansion not in ("heuristic", "residual"):
        raise ValueError("expansion must be 'heuristic' or 'residual'")
    return d3s_sweep_params(alpha, 1 if adaptive else 0, eps, tol, kmax, max_matvecs, prec, e_before, m_limit,
                            mixed_min_gflop, 1 if expansion == "residual" else 0)


# --- symmetry blocks -------------------------------------------------------
def _ints(a):
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32).ravel())
    return arr, arr.ctypes.data_as(c_int_p)


LAYOUT_DENSE, LAYOUT_PACKED = 0, 1


class BlockPlan:
    """Task tables of one block-sparse H_eff (d3s_block_plan_create_layout);
    `layout` LAYOUT_DENSE (tensors in the dense layouts) or LAYOUT_PACKED (only
    the allowed blocks; the sizes are self.nl, self.nr, self.npsi)."""

    def __init__(self, ctx, nq, d, wl, wr, left_q, left_dim, right_q, right_dim, phys_q, wq_left, wq_right,
                 layout=LAYOUT_DENSE):
        self.ctx = ctx
        self.h = None
        self._keep = []

        def sec(q, dim):
            qa, qp = _ints(q)
            da, dp = _ints(dim)
            self._keep += [qa, da]
            return d3s_sectors(len(da), qp, dp)
        self.left, self.right = sec(left_q, left_dim), sec(right_q, right_dim)
        pa, pp = _ints(phys_q)
        la, lp = _ints(wq_left)
        ra, rp = _ints(wq_right)
        self._keep += [pa, la, ra]
        self.ml, self.mr = int(sum(left_dim)), int(sum(right_dim))
        self.d, self.wl, self.wr, self.nq = d, wl, wr, nq
        h = c_void_p()
        fl = c_double()
        nt = c_int()
        ctx._sync_stream()
        ctx._check(_plan_create_layout(ctx.h, nq, d, wl, wr, ctypes.byref(self.left), ctypes.byref(self.right), pp,
                                       lp, rp, int(layout), ctypes.byref(h), ctypes.byref(fl), ctypes.byref(nt)))
        self.h = h
        self.layout = int(layout)
        self.flops = fl.value
        self.ntasks = nt.value
        ctx._plans.add(self)
        nl, nr, npsi = c_long(), c_long(), c_long()
        ctx._check(_plan_sizes(h, ctypes.byref(nl), ctypes.byref(nr), ctypes.byref(npsi)))
        self.nl, self.nr, self.npsi = nl.value, nr.value, npsi.value

    def bind(self, L, W, R, prec):
        """d3s_block_plan_bind: FP64 L, W, R (the plan's layout) converted for
        FP32 / BF16 products held by the plan."""
        ctx = self.ctx
        ctx._sync_stream()
        f = torch.float64
        _need(L, self.nl, f, "L")
        _need(W, self.wl * self.wr * self.d * self.d, f, "W")
        _need(R, self.nr, f, "R")
        return ctx._check(_plan_bind(ctx.h, self.h, int(prec), _ptr(L), _ptr(W), _ptr(R)))

    def apply_bound(self, psi, out, use_graph=False):
        """d3s_apply_heff_blocks_bound: out = H psi (FP64, the plan's layout)
        with the bound operator."""
        ctx = self.ctx
        ctx._sync_stream()
        _need(psi, self.npsi, torch.float64, "psi")
        _need(out, self.npsi, torch.float64, "out")
        return ctx._check(_apply_bound(ctx.h, self.h, _ptr(psi), _ptr(out), 1 if use_graph else 0))

    def apply(self, L, W, R, psi, out, use_graph=False):
        ctx = self.ctx
        ctx._sync_stream()
        ml, d, mr, wl, wr = self.ml, self.d, self.mr, self.wl, self.wr
        prec = _PREC[psi.dtype]
        te, tw, to = _ELT[prec]
        _need(L, self.nl, te, "L")
        _need(W, wl * wr * d * d, tw, "W")
        _need(R, self.nr, te, "R")
        _need(psi, self.npsi, te, "psi")
        _need(out, self.npsi, to, "out")
        return ctx._check(_apply_blocks(ctx.h, self.h, prec, _ptr(L), _ptr(W), _ptr(R), _ptr(psi), _ptr(out),
                                        1 if use_graph else 0))

    def expand_subspace(self, direction, env, W, psi, alpha, Mtilde):
        """Block-sparse d3s_expand_subspace (FP64) on the plan's bonds."""
        ctx = self.ctx
        ctx._sync_stream()
        ml, d, mr, wl, wr = self.ml, self.d, self.mr, self.wl, self.wr
        f = torch.float64
        _need(W, wl * wr * d * d, f, "W")
        _need(psi, ml * d * mr, f, "psi")
        if direction == L2R:
            _need(env, ml * wl * ml, f, "L")
            _need(Mtilde, ml * d * (1 + wr) * mr, f, "Mtilde")
        else:
            _need(env, mr * wr * mr, f, "R")
            _need(Mtilde, (1 + wl) * ml * d * mr, f, "Mtilde")
        return ctx._check(_expand_blocks(ctx.h, self.h, direction, _ptr(env), _ptr(W), _ptr(psi), float(alpha),
                                         _ptr(Mtilde)))

    def truncate(self, direction, Mtilde, psi, kmax, rel_cutoff, nbr, site_out, nbr_out, renormalize=True,
                 maxsec=4096):
        """Block-diagonal d3s_truncate of [psi | alpha P] / [psi ; alpha P] on the
        plan's bonds.  Returns (k, discarded, new sector charges (nsec x nq),
        new sector dims)."""
        import numpy as np
        ctx = self.ctx
        ctx._sync_stream()
        ml, d, mr, wl, wr = self.ml, self.d, self.mr, self.wl, self.wr
        f = torch.float64
        _need(psi, ml * d * mr, f, "psi")
        if direction == L2R:
            other = nbr.numel() // mr
            _need(Mtilde, ml * d * (1 + wr) * mr, f, "Mtilde")
            _need(site_out, ml * d * min(kmax, ml * d), f, "site_out")
        else:
            other = nbr.numel() // ml
            _need(Mtilde, (1 + wl) * ml * d * mr, f, "Mtilde")
            _need(site_out, d * mr * min(kmax, d * mr), f, "site_out")
        _need(nbr_out, min(kmax, ml * d if direction == L2R else d * mr) * other, f, "nbr_out")
        nq = self.nq
        nsec = c_int()
        q = np.zeros(maxsec * nq, dtype=np.int32)
        dims = np.zeros(maxsec, dtype=np.int32)
        k = c_int()
        disc = c_double()
        ctx._check(_trunc_blocks(ctx.h, self.h, direction, _ptr(Mtilde), _ptr(psi), kmax, float(rel_cutoff),
                                 _ptr(nbr), other, _ptr(site_out), _ptr(nbr_out), 1 if renormalize else 0, maxsec,
                                 ctypes.byref(nsec), q.ctypes.data_as(c_int_p), dims.ctypes.data_as(c_int_p),
                                 ctypes.byref(k), ctypes.byref(disc)))
        ns = nsec.value
        return k.value, disc.value, q[: ns * nq].reshape(ns, nq), dims[:ns]

    def update_env(self, direction, env_in, W, site, env_out):
        """Block-sparse d3s_update_env (FP64) for a site tensor on the plan's bonds."""
        ctx = self.ctx
        ctx._sync_stream()
        ml, d, mr, wl, wr = self.ml, self.d, self.mr, self.wl, self.wr
        f = torch.float64
        _need(W, wl * wr * d * d, f, "W")
        _need(site, ml * d * mr, f, "site")
        if direction == L2R:
            _need(env_in, ml * wl * ml, f, "L")
            _need(env_out, mr * wr * mr, f, "env_out")
        else:
            _need(env_in, mr * wr * mr, f, "R")
            _need(env_out, ml * wl * ml, f, "env_out")
        return ctx._check(_env_blocks(ctx.h, self.h, direction, _ptr(env_in), _ptr(W), _ptr(site), _ptr(env_out)))

    def close(self):
        if self.h and self.ctx.h:
            _plan_destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpo_spin_charges(rng):
    import numpy as np
    out = np.zeros(2 + 3 * rng, dtype=np.int32)
    if _spin_charges(rng, out.ctypes.data_as(c_int_p)) != OK:
        raise D3SError(EINVAL, "d3s_mpo_spin_charges")
    return out.reshape(-1, 1)


def mpo_fermion_charges(rng):
    import numpy as np
    out = np.zeros((2 + 4 * rng) * 2, dtype=np.int32)
    if _fermion_charges(rng, out.ctypes.data_as(c_int_p)) != OK:
        raise D3SError(EINVAL, "d3s_mpo_fermion_charges")
    return out.reshape(-1, 2)


SPIN_HALF_CHARGES = [[1], [-1]]                          # 2Sz of |up>, |down>
HUBBARD_CHARGES = [[0, 0], [1, 1], [1, -1], [2, 0]]      # (N, 2Sz) of |0>, |up>, |dn>, |updn>


# --- model builders (host) -------------------------------------------------
def _blocks(flat, offsets, dims, l, d):
    out = []
    for i in range(l):
        n = dims[i] * dims[i + 1] * d * d
        out.append(flat[offsets[i]: offsets[i] + n].reshape(dims[i], dims[i + 1], d, d).copy())
    return out


def mpo_spin_exchange(l, J_table):
    """J_table: (l, range) array, J_table[i, r-1] = J_{i, i+r}."""
    import numpy as np
    J = np.ascontiguousarray(J_table, dtype=np.float64)
    rng = J.shape[1]
    total = c_long()
    dims = (c_int * (l + 1))()
    offs = (c_long * l)()
    Jp = J.ctypes.data_as(c_double_p)
    st = _mpo_spin(l, rng, Jp, None, offs, dims, ctypes.byref(total))
    if st != OK:
        raise D3SError(st, "d3s_mpo_spin_exchange")
    flat = np.zeros(total.value)
    _mpo_spin(l, rng, Jp, flat.ctypes.data_as(c_double_p), offs, dims, ctypes.byref(total))
    return _blocks(flat, list(offs), list(dims), l, 2)


def mpo_fermion_hopping(l, t_table, U=0.0, mu=None):
    import numpy as np
    t = np.ascontiguousarray(t_table, dtype=np.float64)
    rng = t.shape[1]
    mu_arr = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
    mup = None if mu_arr is None else mu_arr.ctypes.data_as(c_double_p)
    total = c_long()
    dims = (c_int * (l + 1))()
    offs = (c_long * l)()
    tp = t.ctypes.data_as(c_double_p)
    st = _mpo_fermion(l, rng, tp, float(U), mup, None, offs, dims, ctypes.byref(total))
    if st != OK:
        raise D3SError(st, "d3s_mpo_fermion_hopping")
    flat = np.zeros(total.value)
    _mpo_fermion(l, rng, tp, float(U), mup, flat.ctypes.data_as(c_double_p), offs, dims, ctypes.byref(total))
    return _blocks(flat, list(offs), list(dims), l, 4)


def heisenberg_mpo(l, J=1.0):
    import numpy as np
    return mpo_spin_exchange(l, np.full((l, 1), J))


def j1j2_mpo(l, J1=1.0, J2=0.0):
    import numpy as np
    tab = np.zeros((l, 2))
    tab[:, 0] = J1
    tab[:, 1] = J2
    return mpo_spin_exchange(l, tab)


def hubbard_chain_mpo(l, t=1.0, U=0.0, mu=None):
    import numpy as np
    return mpo_fermion_hopping(l, np.full((l, 1), t), U=U, mu=mu)


def hubbard_cylinder_mpo(width, length, t=1.0, U=0.0):
    """Sites numbered column by column (s = x*width + y), periodic across the
    width; every column traversed in the same direction (hopping range = width)."""
    import numpy as np
    l = width * length
    tab = np.zeros((l, width))
    for x in range(length):
        for y in range(width):
            s = x * width + y
            if width > 1 and (y + 1 < width or width > 2):
                s2 = x * width + (y + 1) % width
                i, j = min(s, s2), max(s, s2)
                tab[i, j - i - 1] = t
            if x + 1 < length:
                tab[s, width - 1] = t
    return mpo_fermion_hopping(l, tab, U=U)
