"""Python face of the chebtd C ABI, with torch tensors for device memory.

Each method forwards to the entry point of the same name in
include/chebtd.h.  Tensors must live on the context's GPU, be contiguous and
have the dtype stated (complex128 states, float64 potentials); they are
checked here before their pointers cross the boundary.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

_EDGES = {"zigzag": L.ZIGZAG, "armchair": L.ARMCHAIR}


def _torch():
    import torch
    return torch


def _need(t, dtype, n=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def holstein_csr_host(L_sites: int, nph: int, t: float, w0: float, g, Delta, periodic: bool):
    """CSR of eq. (ghm) built by the library's host code (no GPU needed)."""
    lib = L.lib()
    g = np.ascontiguousarray(np.broadcast_to(np.asarray(g, float), (L_sites,)), dtype=np.float64)
    D = np.ascontiguousarray(np.broadcast_to(np.asarray(Delta, float), (L_sites,)), dtype=np.float64)
    n, nnz = C.c_int64(), C.c_int64()
    gp, dp = g.ctypes.data_as(C.c_void_p), D.ctypes.data_as(C.c_void_p)
    L.check(lib.chebtd_holstein_csr_host(L_sites, nph, t, w0, gp, dp, int(periodic), C.byref(n),
                                         C.byref(nnz), None, None, None))
    rowptr = np.zeros(n.value + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.complex128)
    L.check(lib.chebtd_holstein_csr_host(L_sites, nph, t, w0, gp, dp, int(periodic), C.byref(n),
                                         C.byref(nnz), rowptr.ctypes.data_as(C.c_void_p),
                                         col.ctypes.data_as(C.c_void_p),
                                         val.ctypes.data_as(C.c_void_p)))
    return rowptr, col, val


def holstein_occupations(L_sites: int, nph: int) -> np.ndarray:
    lib = L.lib()
    cnt = C.c_int64()
    L.check(lib.chebtd_holstein_occupations(L_sites, nph, C.byref(cnt), None))
    occ = np.zeros(cnt.value * L_sites, dtype=np.uint8)
    L.check(lib.chebtd_holstein_occupations(L_sites, nph, C.byref(cnt),
                                            occ.ctypes.data_as(C.c_void_p)))
    return occ.reshape(cnt.value, L_sites)


def region_sum_noalloc(psi, mask, out, stream=None):
    """sum_i mask_i |psi_i|^2 into out[0] without any device allocation (the
    library's fixed per-GPU scratch; chebtd_region_sum_noalloc).  psi:
    complex128, mask: uint8, out: float64 CUDA tensors the caller owns;
    stream: a torch stream (default: the current one)."""
    torch = _torch()
    n = psi.numel()
    p = _need(psi, torch.complex128, n, "psi")
    m = _need(mask, torch.uint8, n, "mask")
    o = _need(out, torch.float64, None, "out")
    if out.numel() < 1:
        raise ValueError("out must hold one value")
    st = stream if stream is not None else torch.cuda.current_stream(psi.device)
    L.check(L.lib().chebtd_region_sum_noalloc(p, m, n, o, C.c_void_p(st.cuda_stream)))
    return out


class Context:
    """A chebtd context on the current GPU and torch stream."""

    def __init__(self, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise L.ChebError(L.E_STATE, "no GPU visible: chebtd runs only on the GPU")
        self._lib = L.lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = self._lib.chebtd_create(C.byref(h), C.c_void_p(stream.cuda_stream))
        L.check(rc, None)
        self.h = h
        self._keep = {}   # borrowed device arrays of the current Hamiltonian
        self._bkeep = []  # borrowed arrays of the batch
        self.n = 0

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self._lib.chebtd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        L.check(rc, self.h)

    # -- Hamiltonians -------------------------------------------------------
    def chain1d(self, V, dx: float):
        torch = _torch()
        p = _need(V, torch.float64, name="V")
        self._check(self._lib.chebtd_h_chain1d(self.h, V.numel(), float(dx), p))
        self._keep = {"V": V}
        self.n = V.numel()
        return self

    def honeycomb(self, width: int, length: int, eps, edge: str = "zigzag", t: float = 1.0):
        torch = _torch()
        p = _need(eps, torch.float64, width * length, "eps")
        self._check(self._lib.chebtd_h_honeycomb(self.h, width, length, _EDGES[edge], float(t), p))
        self._keep = {"eps": eps}
        self.n = width * length
        return self

    def csr(self, rowptr, col, val):
        torch = _torch()
        n = rowptr.numel() - 1
        pr = _need(rowptr, torch.int64, name="rowptr")
        pc = _need(col, torch.int32, name="col")
        pv = _need(val, torch.complex128, col.numel(), "val")
        self._check(self._lib.chebtd_h_csr(self.h, n, col.numel(), pr, pc, pv))
        self._keep = {"rowptr": rowptr, "col": col, "val": val}
        self.n = n
        return self

    def holstein(self, L_sites: int, nph: int, t: float, w0: float, g, Delta, periodic: bool):
        g = np.ascontiguousarray(np.broadcast_to(np.asarray(g, float), (L_sites,)), dtype=np.float64)
        D = np.ascontiguousarray(np.broadcast_to(np.asarray(Delta, float), (L_sites,)),
                                 dtype=np.float64)
        self._check(self._lib.chebtd_h_holstein(self.h, L_sites, nph, float(t), float(w0),
                                                g.ctypes.data_as(C.c_void_p),
                                                D.ctypes.data_as(C.c_void_p), int(periodic)))
        self._keep = {}
        self.n = int(self._lib.chebtd_dim(self.h))
        self.hol_L = L_sites
        return self

    # -- bounds and plan ------------------------------------------------------
    def gershgorin(self):
        lo, hi = C.c_double(), C.c_double()
        self._check(self._lib.chebtd_gershgorin(self.h, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def set_bounds(self, emin: float, emax: float, alpha: float = 0.01):
        self._check(self._lib.chebtd_set_bounds(self.h, float(emin), float(emax), float(alpha)))
        return self

    def plan(self, dt: float, tol: float = 1e-15) -> int:
        M = C.c_int()
        self._check(self._lib.chebtd_plan(self.h, float(dt), float(tol), C.byref(M)))
        return M.value

    def plan_order(self, dt: float, M: int):
        self._check(self._lib.chebtd_plan_order(self.h, float(dt), int(M)))
        return self

    def get_plan(self):
        a, b, dt, M = C.c_double(), C.c_double(), C.c_double(), C.c_int()
        self._check(self._lib.chebtd_get_plan(self.h, None, C.byref(a), C.byref(b), C.byref(dt),
                                              C.byref(M)))
        g = np.zeros(M.value + 1, dtype=np.complex128)
        self._check(self._lib.chebtd_get_plan(self.h, g.ctypes.data_as(C.c_void_p), None, None,
                                              None, None))
        return dict(gamma=g, a=a.value, b=b.value, dt=dt.value, M=M.value)

    def plan_passes(self):
        """Orders per pass of one step on the multi-order path ([] when the
        plan runs one order per launch)."""
        n = C.c_int()
        self._check(self._lib.chebtd_plan_passes(self.h, None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        self._check(self._lib.chebtd_plan_passes(self.h, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        return [int(v) for v in out[:n.value]]

    # -- propagation ------------------------------------------------------------
    def propagate(self, psi, K: int, norm=None, energy=None, flags: int = 0):
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        pn = _need(norm, torch.float64, None, "norm") if norm is not None else None
        pe = _need(energy, torch.float64, None, "energy") if energy is not None else None
        if norm is not None and norm.numel() < K:
            raise ValueError("norm needs K entries")
        if energy is not None and energy.numel() < K:
            raise ValueError("energy needs K entries")
        self._check(self._lib.chebtd_propagate(self.h, p, int(K), pn, pe, int(flags)))
        return psi

    def propagate_td(self, psi, onsite, norm=None, energy=None, flags: int = 0):
        """K = onsite.shape[0] steps; onsite[s] is the step's V (chain), eps
        (ribbon) or Delta (Holstein)."""
        torch = _torch()
        if onsite.dim() != 2:
            raise ValueError("onsite must be (K, values per step)")
        K = onsite.shape[0]
        p = _need(psi, torch.complex128, self.n, "psi")
        po = _need(onsite, torch.float64, None, "onsite")
        pn = _need(norm, torch.float64, None, "norm") if norm is not None else None
        pe = _need(energy, torch.float64, None, "energy") if energy is not None else None
        for t, nm in ((norm, "norm"), (energy, "energy")):
            if t is not None and t.numel() < K:
                raise ValueError(f"{nm} needs K entries")
        self._check(self._lib.chebtd_propagate_td(self.h, p, int(K), po, int(onsite.shape[1]), pn, pe,
                                                  int(flags)))
        return psi

    def crank_nicolson(self, psi, dt: float, S: int):
        """S Crank-Nicolson steps of the current 1D chain (comparison method)."""
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        self._check(self._lib.chebtd_crank_nicolson(self.h, p, float(dt), int(S)))
        return psi

    def set_check_tol(self, rel_tol: float):
        self._check(self._lib.chebtd_set_check_tol(self.h, float(rel_tol)))

    # -- observables -------------------------------------------------------------
    def density(self, psi, out=None):
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=psi.device)
        self._check(self._lib.chebtd_density(self.h, p, _need(out, torch.float64, self.n, "rho")))
        return out

    def region_sum(self, psi, mask, out=None):
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        m = _need(mask, torch.uint8, self.n, "mask")
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=psi.device)
        self._check(self._lib.chebtd_region_sum(self.h, p, m, _need(out, torch.float64, None, "out")))
        return out

    def norm_energy(self, psi, out=None):
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=psi.device)
        self._check(self._lib.chebtd_norm_energy(self.h, p, _need(out, torch.float64, None, "out")))
        return out

    def holstein_obs(self, psi):
        torch = _torch()
        p = _need(psi, torch.complex128, self.n, "psi")
        Ls = self.hol_L
        n_i = torch.empty(Ls, dtype=torch.float64, device=psi.device)
        nph = torch.empty_like(n_i)
        chi = torch.empty_like(n_i)
        self._check(self._lib.chebtd_holstein_obs(self.h, p, C.c_void_p(n_i.data_ptr()),
                                                  C.c_void_p(nph.data_ptr()),
                                                  C.c_void_p(chi.data_ptr())))
        return n_i, nph, chi

    # -- batched ribbons -----------------------------------------------------------
    def batch_create(self, systems, dt: float, alpha: float = 0.01, tol: float = 1e-15):
        """systems: list of dicts with width, length, eps (cuda f64), psi (cuda c128),
        emin, emax and optional edge ('zigzag'/'armchair') and t."""
        torch = _torch()
        arr = (L.SysDesc * len(systems))()
        keep = []
        for i, s in enumerate(systems):
            n = s["width"] * s["length"]
            arr[i].width = s["width"]
            arr[i].length = s["length"]
            arr[i].edge = _EDGES[s.get("edge", "zigzag")]
            arr[i].t_hop = float(s.get("t", 1.0))
            arr[i].eps_dev = _need(s["eps"], torch.float64, n, "eps").value
            arr[i].emin = float(s["emin"])
            arr[i].emax = float(s["emax"])
            arr[i].psi_dev = _need(s["psi"], torch.complex128, n, "psi").value
            keep += [s["eps"], s["psi"]]
        self._check(self._lib.chebtd_batch_create(self.h, len(systems), arr, float(dt),
                                                  float(alpha), float(tol)))
        self._bkeep = keep
        self._bsizes = [s["width"] * s["length"] for s in systems]
        return self

    def batch_set_schedule(self, mode: int, tile_rows: int, block: int, wg_per_cu: int = 2):
        self._check(self._lib.chebtd_batch_set_schedule(self.h, int(mode), int(tile_rows),
                                                        int(block), int(wg_per_cu)))

    def batch_autotune(self, cache_path: str | None = None):
        best = (C.c_int * 4)()
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.chebtd_batch_autotune(self.h, path, best))
        return tuple(best)

    def batch_propagate(self, K: int, flags: int = 0, psi=None):
        """psi: None (the bound states) or one complex128 CUDA tensor per
        system, propagated in place and bound for later calls."""
        arr = None
        if psi is not None:
            torch = _torch()
            if len(psi) != len(self._bsizes):
                raise ValueError("need one state per system")
            arr = (C.c_void_p * len(psi))()
            for i, (p, n) in enumerate(zip(psi, self._bsizes)):
                arr[i] = _need(p, torch.complex128, n, f"psi[{i}]").value
            self._bkeep = [t for t in self._bkeep[0::2]] + list(psi)
        self._check(self._lib.chebtd_batch_propagate(self.h, arr, int(K), int(flags)))

    def batch_info(self):
        ns = C.c_int()
        self._check(self._lib.chebtd_batch_info(self.h, C.byref(ns), None))
        Ms = np.zeros(ns.value, dtype=np.int32)
        self._check(self._lib.chebtd_batch_info(self.h, C.byref(ns), Ms.ctypes.data_as(C.c_void_p)))
        return Ms

    # -- adjoint ----------------------------------------------------------------------
    def reserve_adjoint(self, max_steps: int, mode: int = L.ADJ_STEP):
        self._check(self._lib.chebtd_reserve_adjoint(self.h, int(max_steps), int(mode)))

    def checkpoint_run(self) -> int:
        """Number of the checkpointing run whose trajectory is stored (0: none)."""
        rid = C.c_int64()
        self._check(self._lib.chebtd_checkpoint_run(self.h, C.byref(rid)))
        return rid.value

    def adjoint(self, gbar, dLdV, run: int | None = None):
        """run: the checkpointing run the gradient is for (checked); None
        takes the stored one."""
        torch = _torch()
        pg = _need(gbar, torch.complex128, self.n, "gbar")
        pd = _need(dLdV, torch.float64, self.n, "dLdV")
        if run is None:
            self._check(self._lib.chebtd_adjoint(self.h, pg, pd))
        else:
            self._check(self._lib.chebtd_adjoint_run(self.h, int(run), pg, pd))

    # -- measurement ---------------------------------------------------------------------
    def time_recursion_kernel(self, launches: int = 100, flags: int = 0):
        """(ms per launch, kernel name, recursion orders per launch)."""
        ms = C.c_double()
        name = C.c_char_p()
        orders = C.c_int()
        self._check(self._lib.chebtd_time_recursion_kernel(self.h, int(launches), int(flags), C.byref(ms),
                                                           C.byref(name), C.byref(orders)))
        return ms.value, name.value.decode(), orders.value
