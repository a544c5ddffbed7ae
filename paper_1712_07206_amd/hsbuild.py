"""PyTorch-facing wrapper of the hsbuild C-ABI.

Only marshalling happens here: tensors are checked for dtype, device and
contiguity, the workspace is a uint8 CUDA tensor, and the library is called
on torch's current stream.  Every step of the computation runs in the HIP
library.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(t.shape)))
    return t.contiguous()


class HSBuilder:
    """One cell (lattice, atom types, radii, radial boundary values) bound to
    the current HIP device.  Inputs per call: k (fractional), the G list,
    atom positions tau and the per-type T blocks."""

    def __init__(self, lattice, atom_type, r_mt, radial, udot_norm2, l_max: int, max_ng: int,
                 precision: int = N.HSB_FP64, n_slices: int = 0):
        self._atom_type = np.ascontiguousarray(atom_type, dtype=np.int32)
        self._r_mt = np.ascontiguousarray(r_mt, dtype=np.float64)
        self._radial = np.ascontiguousarray(radial, dtype=np.float64)
        self._udot = np.ascontiguousarray(udot_norm2, dtype=np.float64)
        lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
        self.n_types = int(self._r_mt.shape[0])
        self.n_atoms = int(self._atom_type.shape[0])
        self.l_max = int(l_max)
        self.n_l = (self.l_max + 1) ** 2
        self.max_ng = int(max_ng)
        cfg = N.HsbConfig()
        cfg.n_types = self.n_types
        cfg.n_atoms = self.n_atoms
        cfg.l_max = self.l_max
        cfg.max_ng = self.max_ng
        for i in range(9):
            cfg.lattice[i] = float(lat[i])
        cfg.atom_type = self._atom_type.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.r_mt = self._r_mt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.radial = self._radial.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.udot_norm2 = self._udot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        cfg.precision = int(precision)
        cfg.n_slices = int(n_slices)
        handle = ctypes.c_void_p()
        code = N.lib().hsbuild_create(ctypes.byref(cfg), ctypes.byref(handle))
        if code != N.HSB_OK:
            raise N.HSBuildError(code, N.last_error(None))
        self._h = handle
        self._ws: Optional[torch.Tensor] = None

    @classmethod
    def from_case(cls, case: dict, max_ng: Optional[int] = None, precision: int = N.HSB_FP64,
                  n_slices: int = 0) -> "HSBuilder":
        if max_ng is None:
            ng = case["n_g"]
            max_ng = int(np.max(ng))
        return cls(case["lattice"], case["atom_type"], case["r_mt"], case["radial"], case["udot_norm2"],
                   case["l_max"], max_ng, precision, n_slices)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().hsbuild_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspace -------------------------------------------------------------------
    def workspace_bytes(self, mode: int, ng: Sequence[int]) -> int:
        arr = (ctypes.c_int32 * len(ng))(*[int(x) for x in ng])
        nbytes = N.lib().hsbuild_workspace_bytes(self._h, int(mode), len(ng), arr)
        if nbytes == 0:
            raise N.HSBuildError(N.HSB_ERR_ARG, N.last_error(self._h))
        return int(nbytes)

    def workspace(self, mode: int, ng: Sequence[int]) -> torch.Tensor:
        need = self.workspace_bytes(mode, ng)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    # -- entry points ------------------------------------------------------------------
    def coefficients(self, k_frac, g: torch.Tensor, tau: torch.Tensor, out: Optional[torch.Tensor] = None):
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        shape = (self.n_atoms, 2, self.n_l, ng)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        out = _dev(out, torch.complex128, "out", shape)
        ws = self.workspace(N.HSB_MODE_COEFFICIENTS, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_coefficients(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(out), _ptr(ws),
                                             ws.numel(), _stream()), self._h)
        return out

    def forward(self, k_frac, g: torch.Tensor, tau: torch.Tensor, T: torch.Tensor,
                H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
        """Upper triangles of H and S (column >= row); the strict lower
        triangle of caller-supplied H, S is left as it was."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        if ws is None:
            ws = self.workspace(N.HSB_MODE_FORWARD, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_forward(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(H), _ptr(S),
                                        _ptr(ws), ws.numel(), _stream()), self._h)
        return H, S

    def forward_static(self, k_frac, g: torch.Tensor, tau: torch.Tensor, T: torch.Tensor,
                       H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None):
        """hsbuild_forward_static: as forward(), with the library's own device
        scratch instead of a workspace (nothing is allocated by the call; H and
        S are allocated here only when not given)."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_forward_static(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(H), _ptr(S),
                                               _stream()), self._h)
        return H, S

    def forward_factored(self, k_frac, g: torch.Tensor, tau: torch.Tensor, T: torch.Tensor,
                         H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None):
        """H and S by the type-factored contraction (hsbuild_forward_factored):
        the same upper triangles as forward, in FP64 whatever the precision."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        if ws is None:
            ws = self.workspace(N.HSB_MODE_FACTORED, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_forward_factored(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(H), _ptr(S),
                                                 _ptr(ws), ws.numel(), _stream()), self._h)
        return H, S

    def forward_hsdla(self, algorithm: int, k_frac, g: torch.Tensor, tau: torch.Tensor, T: torch.Tensor,
                      H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None,
                      ws: Optional[torch.Tensor] = None):
        """H and S by the paper's BLAS sequence on rocBLAS (hsbuild_forward_hsdla):
        algorithm 3 (refined) or 1 (original, H_AA by a full zgemm)."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        if ws is None:
            ws = self.workspace(N.HSB_MODE_HSDLA, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_forward_hsdla(self._h, int(algorithm), kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(H),
                                              _ptr(S), _ptr(ws), ws.numel(), _stream()), self._h)
        return H, S

    def forward_real(self, k_frac, g: torch.Tensor, tau: torch.Tensor, partner, T: torch.Tensor,
                     H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None):
        """Real-symmetric H and S of an inversion-symmetric cell
        (hsbuild_forward_real): float64 upper triangles.  partner[a] is the
        atom at -tau_a (a for an atom at the origin)."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        part = np.ascontiguousarray(np.asarray(partner, dtype=np.int32).reshape(-1))
        if part.shape != (self.n_atoms,):
            raise ValueError("partner must have one entry per atom")
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.float64, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.float64, device="cuda")
        H = _dev(H, torch.float64, "H", (ng, ng))
        S = _dev(S, torch.float64, "S", (ng, ng))
        if ws is None:
            ws = self.workspace(N.HSB_MODE_REAL, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_forward_real(self._h, kf, ng, _ptr(g), _ptr(tau),
                                             part.ctypes.data_as(ctypes.c_void_p), _ptr(T), _ptr(H), _ptr(S),
                                             _ptr(ws), ws.numel(), _stream()), self._h)
        return H, S

    def eigensolve(self, H: torch.Tensor, S: torch.Tensor, vectors: bool = True):
        """Generalized eigenproblem H c = lambda S c (hsbuild_eigensolve) on the
        upper triangles of a forward call, in place: returns (eigenvalues,
        rocSOLVER info); with vectors, row j of H becomes the eigenvector c_j."""
        ng = int(H.shape[0])
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        w = torch.empty(ng, dtype=torch.float64, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = self.workspace(N.HSB_MODE_EIGEN, [ng])
        N.check(N.lib().hsbuild_eigensolve(self._h, ng, _ptr(H), _ptr(S), _ptr(w), 1 if vectors else 0, _ptr(info),
                                           _ptr(ws), ws.numel(), _stream()), self._h)
        return w, int(info.item())

    def backward(self, k_frac, g: torch.Tensor, tau: torch.Tensor, T: torch.Tensor, gH: torch.Tensor,
                 gS: torch.Tensor, gT: Optional[torch.Tensor] = None, gtau: Optional[torch.Tensor] = None):
        """Gradients of a real loss with Hermitian dL/dH = gH and dL/dS = gS
        (torch convention dL/dRe + i dL/dIm): returns (dL/dT, dL/dtau)."""
        ng = int(g.shape[0])
        g = _dev(g, torch.int32, "g", (ng, 3))
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        m = 2 * self.n_l
        T = _dev(T, torch.complex128, "T", (self.n_types, m, m))
        gH = _dev(gH, torch.complex128, "gH", (ng, ng))
        gS = _dev(gS, torch.complex128, "gS", (ng, ng))
        if gT is None:
            gT = torch.empty((self.n_types, m, m), dtype=torch.complex128, device="cuda")
        if gtau is None:
            gtau = torch.empty((self.n_atoms, 3), dtype=torch.float64, device="cuda")
        gT = _dev(gT, torch.complex128, "gT", (self.n_types, m, m))
        gtau = _dev(gtau, torch.float64, "gtau", (self.n_atoms, 3))
        ws = self.workspace(N.HSB_MODE_BACKWARD, [ng])
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        N.check(N.lib().hsbuild_backward(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(gH), _ptr(gS),
                                         _ptr(gT), _ptr(gtau), _ptr(ws), ws.numel(), _stream()), self._h)
        return gT, gtau

    def batch(self, k_frac, g_list: Sequence[torch.Tensor], tau: torch.Tensor, T: torch.Tensor,
              H: Optional[torch.Tensor] = None, S: Optional[torch.Tensor] = None, out_off=None,
              ws: Optional[torch.Tensor] = None):
        """H and S of many k-points in one captured graph (one persistent
        contraction).  Returns flat complex128 buffers H, S and the element
        offsets of each k's N_G x N_G block (upper triangles written)."""
        kf = np.ascontiguousarray(k_frac, dtype=np.float64).reshape(-1, 3)
        n_k = kf.shape[0]
        if len(g_list) != n_k:
            raise ValueError("one G list per k-point")
        ng = np.array([int(x.shape[0]) for x in g_list], dtype=np.int32)
        gkey = tuple(int(x.shape[0]) for x in g_list)
        g_in = [_dev(x, torch.int32, "g", (int(x.shape[0]), 3)) for x in g_list]
        if getattr(self, "_gcat_key", None) == gkey:
            # same sizes: refresh the buffer the captured graph refers to (its address stays, so
            # the graph is still replayed, and it reads the lists as they are now)
            g_cat = self._batch_keep
            torch.cat(g_in, out=g_cat)
        else:
            g_cat = _dev(torch.cat(g_in), torch.int32, "g")
        tau = _dev(tau, torch.float64, "tau", (self.n_atoms, 3))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if out_off is None:
            out_off = np.concatenate([[0], np.cumsum(ng.astype(np.int64) ** 2)[:-1]])
        out_off = np.ascontiguousarray(out_off, dtype=np.int64)
        total = int(max(out_off[k] + int(ng[k]) ** 2 for k in range(n_k)))
        if H is None:
            H = torch.empty(total, dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty(total, dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H")
        S = _dev(S, torch.complex128, "S")
        if H.numel() < total or S.numel() < total:
            raise ValueError("H and S need %d elements" % total)
        if ws is None:
            ws = self.workspace(N.HSB_MODE_BATCH, list(ng))
        self._batch_keep = g_cat  # the captured graph refers to this buffer
        self._gcat_key = gkey
        N.check(N.lib().hsbuild_batch(self._h, n_k, kf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      ng.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(g_cat),
                                      out_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(tau), _ptr(T),
                                      _ptr(H), _ptr(S), _ptr(ws), ws.numel(), _stream()), self._h)
        return H, S, out_off

    def forward_from_coefficients(self, coef: torch.Tensor, T: torch.Tensor, H: Optional[torch.Tensor] = None,
                                  S: Optional[torch.Tensor] = None):
        """H and S (upper triangles) from given coefficients [n_atoms][2][N_L][ng]."""
        ng = int(coef.shape[-1])
        coef = _dev(coef, torch.complex128, "coef", (self.n_atoms, 2, self.n_l, ng))
        T = _dev(T, torch.complex128, "T", (self.n_types, 2 * self.n_l, 2 * self.n_l))
        if H is None:
            H = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        if S is None:
            S = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
        H = _dev(H, torch.complex128, "H", (ng, ng))
        S = _dev(S, torch.complex128, "S", (ng, ng))
        ws = self.workspace(N.HSB_MODE_FORWARD, [ng])
        N.check(N.lib().hsbuild_forward_coefficients(self._h, ng, _ptr(coef), _ptr(T), _ptr(H), _ptr(S), _ptr(ws),
                                                     ws.numel(), _stream()), self._h)
        return H, S

    def set_option(self, option: int, value: int) -> None:
        N.check(N.lib().hsbuild_set_option(self._h, int(option), int(value)), self._h)

    def get_option(self, option: int) -> int:
        v = ctypes.c_int32()
        N.check(N.lib().hsbuild_get_option(self._h, int(option), ctypes.byref(v)), self._h)
        return int(v.value)

    def set_timing(self, enable: bool) -> None:
        N.check(N.lib().hsbuild_set_timing(self._h, 1 if enable else 0), self._h)

    def stage_times(self):
        """(average ms of [coefficients, T products (and split operands), contraction kernels,
        recombination], recorded calls)."""
        ms = (ctypes.c_double * N.HSB_TIMING_STAGES)()
        n = ctypes.c_int32()
        N.check(N.lib().hsbuild_stage_times(self._h, ms, ctypes.byref(n)), self._h)
        return [ms[i] for i in range(N.HSB_TIMING_STAGES)], int(n.value)

    def forward_raw(self, k_frac, ng: int, g, tau, T, H, S, ws, ws_bytes: int) -> int:
        """Direct call with pointers already validated by the caller (timing loops)."""
        kf = (ctypes.c_double * 3)(*[float(x) for x in k_frac])
        return N.lib().hsbuild_forward(self._h, kf, ng, _ptr(g), _ptr(tau), _ptr(T), _ptr(H), _ptr(S),
                                       _ptr(ws), ws_bytes, _stream())


def mfma_probe(kind: int, blocks: int, iters: int, out: Optional[torch.Tensor] = None):
    """Enqueue the matrix-core rate probe on the current stream; returns the
    operations it executes and the per-thread output buffer."""
    per = 8 if kind == N.HSB_PROBE_FP64 else 4
    if out is None:
        out = torch.empty(blocks * 256 * per, dtype=torch.uint8, device="cuda")
    ops = ctypes.c_double(0.0)
    code = N.lib().hsbuild_mfma_probe(int(kind), int(blocks), int(iters), _ptr(out), out.numel() * out.element_size(),
                                      _stream(), ctypes.byref(ops))
    N.check(code, None)
    return ops.value, out


def hermitian_full(upper: torch.Tensor) -> torch.Tensor:
    """Full Hermitian matrix from its upper triangle (test and reporting helper)."""
    up = torch.triu(upper)
    return up + torch.triu(upper, 1).conj().transpose(-2, -1)


def case_tensors(case: dict, device="cuda"):
    """Device tensors of a generator case: g, tau, T."""
    g = torch.as_tensor(np.ascontiguousarray(case["g"], dtype=np.int32), device=device)
    tau = torch.as_tensor(np.ascontiguousarray(case["tau"]), device=device)
    T = torch.as_tensor(np.ascontiguousarray(case["T"]), device=device)
    return g, tau, T
