"""torch binding of include/vp_batch.h: a batched slot of resource-block
groups with uneven user counts, run as one captured HIP graph.

`Batch` owns the plan and the device buffers bound to it (inputs H, s;
outputs x, l, cost), laid out group after group as vp_batch.h describes.
Arithmetic runs in the HIP kernels; this module marshals tensors.
"""
from __future__ import annotations

import ctypes
from typing import List, NamedTuple, Optional, Sequence

import torch

from . import _lib
from ._lib import VP_INCLUDE_ZERO, check
from .vp import _stream, packed_size

__all__ = ["GroupSpec", "Batch"]

_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float


class _Group(ctypes.Structure):
    _fields_ = [("n_users", ctypes.c_int32), ("n_sc", ctypes.c_int32), ("K", ctypes.c_int32),
                ("tau", ctypes.c_float), ("alpha", ctypes.c_float)]


class _Info(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("n_sc", ctypes.c_int32), ("n_vec", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("persistent_workgroups", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("class_K", ctypes.c_int32 * 8), ("class_vt", ctypes.c_int32 * 8),
                ("class_pl", ctypes.c_int32 * 8), ("lpt_order", ctypes.c_int32), ("default_ms", ctypes.c_float),
                ("tuned_ms", ctypes.c_float)]


SIGNATURES = {
    "vp_batch_create": [ctypes.POINTER(_Group), _I, _I, _I, _F, ctypes.c_uint32, _P, _P, _P, _P, _P,
                        ctypes.POINTER(_P)],
    "vp_batch_run": [_P, _P],
    "vp_batch_tune": [_P, _I, _P],
    "vp_batch_get_info": [_P, ctypes.POINTER(_Info)],
    "vp_batch_buffers": [_P] + [ctypes.POINTER(_P)] * 6,
    "vp_batch_destroy": [_P],
}
_bound = False


def _load():
    global _bound
    lib = _lib.load()
    if not _bound:
        for name, argtypes in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = argtypes
            fn.restype = _I
        _bound = True
    return lib


class GroupSpec(NamedTuple):
    n_users: int
    n_sc: int
    K: int
    tau: float
    alpha: float


class _DevArray:
    """A device pointer of the plan exposed to torch without a copy."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


_TYPESTR = {torch.complex64: "<c8", torch.float32: "<f4", torch.uint8: "|u1", torch.int32: "<i4"}


def _device_view(ptr: int, n: int, dtype, dev) -> torch.Tensor:
    """A torch view of n elements at device address ptr (no copy)."""
    if n == 0:
        return torch.empty(0, dtype=dtype, device=dev)
    return torch.as_tensor(_DevArray(ptr, (n,), _TYPESTR[dtype]), device=dev)


class Batch:
    """One slot's groups, their bound buffers and the captured plan."""

    def __init__(self, groups: Sequence[GroupSpec], n_t: int, n_sym: int, P_T: float = 0.0,
                 flags: int = VP_INCLUDE_ZERO, device: str = "cuda:0"):
        self.lib = _load()
        self.groups = [GroupSpec(*g) for g in groups]
        self.n_t, self.n_sym, self.P_T = int(n_t), int(n_sym), float(P_T)
        self.dev = torch.device(device)
        self.sizes = [(g.n_users, g.n_sc, g.n_sc * self.n_sym) for g in self.groups]
        nH = sum(g.n_sc * g.n_users * self.n_t for g in self.groups)
        nS = sum(u * nv for u, _, nv in self.sizes)
        self.n_vec = sum(nv for _, _, nv in self.sizes)
        self.n_sc = sum(g.n_sc for g in self.groups)
        self.H = torch.zeros(nH, dtype=torch.complex64, device=self.dev)
        self.s = torch.zeros(nS, dtype=torch.complex64, device=self.dev)
        self.x = torch.empty((self.n_vec, self.n_t), dtype=torch.complex64, device=self.dev)
        self.l = torch.empty((nS, 2), dtype=torch.int8, device=self.dev)
        self.cost = torch.empty(self.n_vec, dtype=torch.float32, device=self.dev)
        arr = (_Group * len(self.groups))(*[_Group(g.n_users, g.n_sc, g.K, g.tau, g.alpha) for g in self.groups])
        plan = _P()
        with torch.cuda.device(self.dev):
            check(self.lib.vp_batch_create(arr, len(self.groups), self.n_t, self.n_sym, self.P_T, int(flags),
                                           self.H.data_ptr(), self.s.data_ptr(), self.x.data_ptr(),
                                           self.l.data_ptr(), self.cost.data_ptr(), ctypes.byref(plan)),
                  "vp_batch_create")
        self.plan = plan
        # offsets of each group in the concatenated arrays
        self._offH, self._offS, self._offV, self._offSc = [], [], [], []
        oh = os_ = ov = osc = 0
        for g, (u, nsc, nv) in zip(self.groups, self.sizes):
            self._offH.append(oh)
            self._offS.append(os_)
            self._offV.append(ov)
            self._offSc.append(osc)
            oh += nsc * u * self.n_t
            os_ += u * nv
            ov += nv
            osc += nsc

    # -- data -----------------------------------------------------------------
    def set_inputs(self, H_list: List, s_list: List):
        """Copy per-group inputs (H [n_sc][N][n_t], s [N][n_vec]; numpy or torch)
        into the bound buffers."""
        for gi, (u, nsc, nv) in enumerate(self.sizes):
            h = torch.as_tensor(H_list[gi]).reshape(-1).to(self.dev, torch.complex64)
            sv = torch.as_tensor(s_list[gi]).reshape(-1).to(self.dev, torch.complex64)
            self.H[self._offH[gi]:self._offH[gi] + h.numel()].copy_(h)
            self.s[self._offS[gi]:self._offS[gi] + sv.numel()].copy_(sv)

    def group_outputs(self, gi: int):
        """(l [N][n_vec][2] int8, cost [n_vec], x [n_vec][n_t]) views of group gi."""
        u, nsc, nv = self.sizes[gi]
        o = self._offS[gi]
        l = self.l[o:o + u * nv].view(u, nv, 2)
        return l, self.cost[self._offV[gi]:self._offV[gi] + nv], self.x[self._offV[gi]:self._offV[gi] + nv]

    def buffers(self):
        """The plan's intermediate arrays as torch views (read-only use)."""
        ptrs = [_P() for _ in range(6)]
        check(self.lib.vp_batch_buffers(self.plan, *[ctypes.byref(p) for p in ptrs]), "vp_batch_buffers")
        nW = sum(nsc * packed_size(u) for u, nsc, _ in self.sizes)
        nN = sum(nsc * u for u, nsc, _ in self.sizes)
        nG = sum(nsc * self.n_t * u for u, nsc, _ in self.sizes)
        nP = sum(g.n_sc * g.K * g.n_users for g in self.groups)

        W = _device_view(ptrs[0].value, nW, torch.complex64, self.dev)
        w2 = _device_view(ptrs[1].value, nN, torch.float32, self.dev)
        perm = _device_view(ptrs[2].value, nN, torch.uint8, self.dev)
        G = _device_view(ptrs[3].value, nG, torch.complex64, self.dev)
        status = _device_view(ptrs[4].value, self.n_sc, torch.int32, self.dev)
        paths = _device_view(ptrs[5].value, nP, torch.uint8, self.dev)
        return {"W": W, "w2": w2, "perm": perm, "G": G, "status": status, "paths": paths}

    def group_buffers(self, gi: int, bufs=None):
        """Per-group views of the intermediate arrays (W, w2, perm, G, status, paths)."""
        bufs = bufs or self.buffers()
        oW = oN = oG = oP = 0
        for j in range(gi):
            u, nsc, _ = self.sizes[j]
            oW += nsc * packed_size(u)
            oN += nsc * u
            oG += nsc * self.n_t * u
            oP += nsc * self.groups[j].K * u
        u, nsc, _ = self.sizes[gi]
        K = self.groups[gi].K
        return {"W": bufs["W"][oW:oW + nsc * packed_size(u)].view(nsc, packed_size(u)),
                "w2": bufs["w2"][oN:oN + nsc * u].view(nsc, u),
                "perm": bufs["perm"][oN:oN + nsc * u].view(nsc, u),
                "G": bufs["G"][oG:oG + nsc * self.n_t * u].view(nsc, self.n_t, u),
                "status": bufs["status"][self._offSc[gi]:self._offSc[gi] + nsc],
                "paths": bufs["paths"][oP:oP + nsc * K * u].view(nsc, K, u)}

    # -- execution ------------------------------------------------------------
    def run(self):
        check(self.lib.vp_batch_run(self.plan, _stream()), "vp_batch_run")

    def tune(self, reps: int = 3):
        check(self.lib.vp_batch_tune(self.plan, int(reps), _stream()), "vp_batch_tune")
        return self.info()

    def info(self) -> dict:
        i = _Info()
        check(self.lib.vp_batch_get_info(self.plan, ctypes.byref(i)), "vp_batch_get_info")
        n = i.n_classes
        return {"n_groups": i.n_groups, "n_sc": i.n_sc, "n_vec": i.n_vec, "n_tiles": i.n_tiles,
                "persistent_workgroups": i.persistent_workgroups,
                "classes": [{"K": i.class_K[c], "vectors_per_tile": i.class_vt[c], "paths_per_lane": i.class_pl[c]}
                            for c in range(n)],
                "lpt_order": bool(i.lpt_order), "default_ms": i.default_ms, "tuned_ms": i.tuned_ms}

    def close(self):
        if getattr(self, "plan", None):
            self.lib.vp_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
