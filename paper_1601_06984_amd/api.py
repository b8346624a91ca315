"""Plan and Sim: thin wrappers over the C ABI (include/mlbm.h)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, lib

_STENCILS = {"D2Q9": _lib.D2Q9, "D3Q19": _lib.D3Q19, "D3Q27": _lib.D3Q27}
_PRECISIONS = {"f64": _lib.F64, "f32": _lib.F32, "f16s": _lib.F16S}


def set_gfc_layers(layers: int = 2):
    """GhostFromCoarser layers of plans created afterwards: 2 (acoustic
    scaling) or 4 (diffusive scaling; such plans have no GPU schedule yet)."""
    check(lib().mlbm_set_gfc_layers(int(layers)))


def lattice(stencil: str):
    """(c (q, d) int, w (q,) float64) of the library's velocity set."""
    s = _STENCILS[stencil]
    q = C.c_int32()
    check(lib().mlbm_lattice(s, C.byref(q), None, None))
    d = 2 if s == _lib.D2Q9 else 3
    c = np.zeros((q.value, d), dtype=np.int32)
    w = np.zeros(q.value, dtype=np.float64)
    check(lib().mlbm_lattice(s, None, c.ctypes.data_as(_lib._pi32), w.ctypes.data_as(_lib._pd)))
    return c, w


def set_morton_policy(level_min_fraction: float = 0.0, block_min_directions: int = 6):
    """Policy for Morton directions of the device pull table in plans created
    afterwards (mlbm_set_morton_policy); the defaults restore the library's."""
    check(lib().mlbm_set_morton_policy(float(level_min_fraction), int(block_min_directions)))


def _i32arr(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int32))
    return a, a.ctypes.data_as(_lib._pi32)


class Plan:
    """Host-only mesh analysis: level-wise element lists and index tables."""

    def __init__(self, stencil: str, level0: int, box_origin, box_extent, face_bc,
                 leaf_ids, solid_ids=()):
        self.stencil = stencil
        self.d = 2 if stencil == "D2Q9" else 3
        self.q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}[stencil]
        self._h = C.c_void_p()
        o, po = _i32arr(box_origin)
        e, pe = _i32arr(box_extent)
        f, pf = _i32arr([_lib.FACE[k] if isinstance(k, str) else int(k) for k in face_bc])
        leaves = np.ascontiguousarray(np.asarray(leaf_ids, dtype=np.uint64))
        solids = np.ascontiguousarray(np.asarray(solid_ids, dtype=np.uint64))
        check(lib().mlbm_plan_create(
            _STENCILS[stencil], int(level0), po, pe, pf,
            leaves.ctypes.data_as(_lib._pu64), len(leaves),
            solids.ctypes.data_as(_lib._pu64) if len(solids) else None, len(solids),
            C.byref(self._h)))
        n = C.c_int32()
        l0 = C.c_int32()
        check(lib().mlbm_plan_levels(self._h, C.byref(n), C.byref(l0)))
        self.n_levels, self.level0 = n.value, l0.value
        g = C.c_int32()
        check(lib().mlbm_plan_gfc_layers(self._h, C.byref(g)))
        self.gfc_layers = g.value
        self._read_info()

    def _read_info(self):
        self.info = []
        for k in range(self.n_levels):
            buf = np.zeros(len(_lib.INFO_FIELDS), dtype=np.int64)
            check(lib().mlbm_plan_level_info(self._h, k, buf.ctypes.data_as(_lib._pi64)))
            self.info.append(dict(zip(_lib.INFO_FIELDS, (int(v) for v in buf))))

    def set_walls(self, ids, dirs, q):
        """Wall fractions of links into solid cells (linear interpolated
        bounce-back): fluid leaf treeIDs, lattice directions pointing into
        the solid (this library's order) and fractions in [0, 1].  Applies
        to simulations created afterwards."""
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32))
        q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
        if not (len(ids) == len(dirs) == len(q)):
            raise ValueError("set_walls: arrays of different lengths")
        n = len(ids)
        check(lib().mlbm_plan_set_walls(
            self._h, ids.ctypes.data_as(_lib._pu64) if n else None,
            dirs.ctypes.data_as(_lib._pi32) if n else None,
            q.ctypes.data_as(_lib._pd) if n else None, n))
        self._read_info()

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.stencil, spec.level0, spec.box_origin, spec.box_extent,
                   spec.face_bc, spec.leaf_ids, spec.solid_ids)

    @property
    def handle(self):
        return self._h

    def export(self, k: int, table: str) -> np.ndarray:
        tid = {"treeid": _lib.TABLE_TREEID, "coords": _lib.TABLE_COORDS,
               "nbr": _lib.TABLE_NBR, "gfc_src": _lib.TABLE_GFC_SRC,
               "gff_src": _lib.TABLE_GFF_SRC, "capture": _lib.TABLE_CAPTURE,
               "bounce": _lib.TABLE_BOUNCE, "nbr16": _lib.TABLE_NBR16,
               "nbase": _lib.TABLE_NBASE, "nbr_wide": _lib.TABLE_NBR_WIDE,
               "nbr_hdr": _lib.TABLE_NBR_HDR, "wall": _lib.TABLE_WALL,
               "wall_q": _lib.TABLE_WALL_Q}[table]
        nbytes = C.c_size_t()
        check(lib().mlbm_plan_export(self._h, k, tid, None, C.byref(nbytes)))
        dtype = {"treeid": np.uint64, "nbr16": np.uint16, "nbr_wide": np.uint16,
                 "wall_q": np.float64}.get(table, np.int32)
        out = np.zeros(nbytes.value // np.dtype(dtype).itemsize, dtype=dtype)
        check(lib().mlbm_plan_export(self._h, k, tid, out.ctypes.data_as(C.c_void_p),
                                     C.byref(nbytes)))
        n = self.info[k]["n"]
        rows = {"coords": self.d, "nbr": self.q - 1, "gfc_src": 4, "gff_src": 4, "bounce": 2,
                "nbr16": self.q - 1, "nbr_wide": self.q - 1}
        if table in rows:
            out = out.reshape(rows[table], -1)
        if table == "wall":
            out = out.reshape(-1, 4)
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().mlbm_plan_destroy(h)
            except Exception:   # interpreter shutdown: modules already torn down
                pass
            self._h = C.c_void_p()


class Sim:
    """A simulation on the current HIP device; memory from torch."""

    def __init__(self, plan: Plan, precision: str = "f32", tau0: float = 0.8,
                 rho0: float = 1.0, u_in=None, f16_exp=None, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("mlbm.Sim needs a HIP device")
        self.torch = torch
        self.plan = plan
        self.precision = precision
        self.device = torch.device(device or "cuda")
        self.stream = stream or torch.cuda.current_stream(self.device)
        need = C.c_size_t()
        check(lib().mlbm_sim_workspace_bytes(plan.handle, _PRECISIONS[precision],
                                             C.byref(need)))
        ws = torch.empty(need.value + 256, dtype=torch.uint8, device=self.device)
        shift = (-ws.data_ptr()) % 256
        self.workspace = ws
        self._ws_ptr = ws.data_ptr() + shift
        self.workspace_bytes = need.value
        uin = None
        if u_in is not None:
            self._uin = np.ascontiguousarray(np.asarray(u_in, dtype=np.float64))
            uin = self._uin.ctypes.data_as(_lib._pd)
        f16 = None
        if f16_exp is not None:
            self._f16 = np.ascontiguousarray(np.asarray(f16_exp, dtype=np.int32))
            f16 = self._f16.ctypes.data_as(_lib._pi32)
        self._h = C.c_void_p()
        check(lib().mlbm_sim_create(plan.handle, _PRECISIONS[precision], float(tau0),
                                    float(rho0), uin, f16, C.c_void_p(self.stream.cuda_stream),
                                    C.c_void_p(self._ws_ptr), need.value, C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def _ptr(self, t, dtype=None):
        if t is None:
            return None
        torch = self.torch
        assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous"
        if dtype is not None:
            assert t.dtype == dtype, f"expected {dtype}, got {t.dtype}"
        return C.c_void_p(t.data_ptr())

    def init(self, k: int, rho, u, S=None):
        """rho (n_fluid,), u (d, n_fluid), S (d(d+1)/2, n_fluid): float64
        device tensors in layout order, S in level-k lattice units."""
        f64 = self.torch.float64
        nf = self.plan.info[k]["n_fluid"]
        ns = 6 if self.plan.d == 3 else 3
        if not 0 <= k < self.plan.n_levels:
            raise ValueError("level index out of range")
        if rho.numel() != nf or u.numel() != self.plan.d * nf or \
                (S is not None and S.numel() != ns * nf):
            raise ValueError(f"level {k}: expected rho[{nf}], u[{self.plan.d}][{nf}], "
                             f"S[{ns}][{nf}]")
        if not hasattr(self, "inputs"):
            self.inputs = {}
        self.inputs[k] = (rho, u, S)
        check(lib().mlbm_init(self._h, k, self._ptr(rho, f64), self._ptr(u, f64),
                              self._ptr(S, f64)))

    def fill_ghosts(self):
        check(lib().mlbm_fill_ghosts(self._h))

    def step(self, n: int = 1):
        check(lib().mlbm_step(self._h, int(n)))

    def diagnostics(self, mask: int = _lib.DIAG_MASS | _lib.DIAG_KE, out=None):
        n = (1 if mask & 1 else 0) + (1 if mask & 2 else 0) + (self.plan.d if mask & 4 else 0)
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        if out.numel() < n:
            raise ValueError("diagnostics output too small")
        check(lib().mlbm_diagnostics(self._h, mask, self._ptr(out, self.torch.float64)))
        return out

    def diagnostics_noalloc(self, mask: int, out):
        """As diagnostics, into the preallocated device tensor `out`, with
        the library's static scratch (allocates nothing)."""
        n = (1 if mask & 1 else 0) + (1 if mask & 2 else 0) + (self.plan.d if mask & 4 else 0)
        if out.numel() < n:
            raise ValueError("diagnostics output too small")
        check(lib().mlbm_diagnostics_noalloc(self._h, mask, self._ptr(out, self.torch.float64)))
        return out

    def get_pdf(self, k: int):
        n = self.plan.info[k]["n"]
        out = self.torch.empty((self.plan.q, n), dtype=self.torch.float64, device=self.device)
        check(lib().mlbm_get_state(self._h, k, _lib.STATE_PDF_POST, self._ptr(out)))
        return out

    def get_moments(self, k: int):
        nf = self.plan.info[k]["n_fluid"]
        out = self.torch.empty((1 + self.plan.d, nf), dtype=self.torch.float64, device=self.device)
        check(lib().mlbm_get_state(self._h, k, _lib.STATE_MOMENTS, self._ptr(out)))
        return out

    def get_pdf_pre(self, k: int):
        """Pre-collision pdfs [q][n_fluid] of the level's fluid elements, as
        its last stream-collide gathered them."""
        nf = self.plan.info[k]["n_fluid"]
        out = self.torch.empty((self.plan.q, nf), dtype=self.torch.float64, device=self.device)
        check(lib().mlbm_get_state(self._h, k, _lib.STATE_PDF_PRE, self._ptr(out)))
        return out

    def get_strain(self, k: int):
        """Strain rate [d(d+1)/2][n_fluid] (xx, yy[, zz], xy[, yz, xz]) of the
        fluid elements from their pre-collision pdfs, level-k lattice units."""
        nf = self.plan.info[k]["n_fluid"]
        ns = 6 if self.plan.d == 3 else 3
        out = self.torch.empty((ns, nf), dtype=self.torch.float64, device=self.device)
        check(lib().mlbm_get_state(self._h, k, _lib.STATE_STRAIN, self._ptr(out)))
        return out

    def get_pdf_prev(self, k: int):
        """The post-collision state [q][n] the level's last stream-collide read."""
        n = self.plan.info[k]["n"]
        out = self.torch.empty((self.plan.q, n), dtype=self.torch.float64, device=self.device)
        check(lib().mlbm_get_state(self._h, k, _lib.STATE_PDF_PREV, self._ptr(out)))
        return out

    def set_pdf(self, k: int, pdf):
        """Overwrite the post-collision pdfs [q][n] of every element."""
        if pdf.numel() != self.plan.q * self.plan.info[k]["n"]:
            raise ValueError("set_pdf expects [q][n] float64")
        check(lib().mlbm_set_state(self._h, k, _lib.STATE_PDF_POST,
                                   self._ptr(pdf, self.torch.float64)))

    def set_pdf_pre(self, k: int, pdf):
        """Collide given pre-collision pdfs [q][n_fluid] of the fluid elements
        into the level's state (sources record their moments)."""
        if pdf.numel() != self.plan.q * self.plan.info[k]["n_fluid"]:
            raise ValueError("set_pdf_pre expects [q][n_fluid] float64")
        check(lib().mlbm_set_state(self._h, k, _lib.STATE_PDF_PRE,
                                   self._ptr(pdf, self.torch.float64)))

    def status(self) -> int:
        f = C.c_uint32()
        check(lib().mlbm_status(self._h, C.byref(f)))
        return f.value

    def time(self) -> int:
        t = C.c_int64()
        check(lib().mlbm_time(self._h, C.byref(t)))
        return t.value

    def checkpoint_bytes(self) -> int:
        b = C.c_size_t()
        check(lib().mlbm_checkpoint_bytes(self._h, C.byref(b)))
        return b.value

    def save_checkpoint(self, buf=None):
        n = self.checkpoint_bytes()
        if buf is None:
            buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        check(lib().mlbm_save_checkpoint(self._h, self._ptr(buf), buf.numel()))
        return buf

    def load_checkpoint(self, buf):
        check(lib().mlbm_load_checkpoint(self._h, self._ptr(buf), buf.numel()))

    def use_graphs(self, enable: bool):
        check(lib().mlbm_use_graphs(self._h, 1 if enable else 0))

    def profile(self, enable: bool):
        check(lib().mlbm_profile(self._h, 1 if enable else 0))

    def profile_read(self, k: int, kind: int = 0):
        """(ms, launches, elements) of level k's stream-collide launches
        (kind 0) or adjoint stream-collide launches (kind 1)."""
        ms, n, el = C.c_double(), C.c_int64(), C.c_int64()
        check(lib().mlbm_profile_read_kind(self._h, kind, k, C.byref(ms), C.byref(n),
                                           C.byref(el)))
        return ms.value, n.value, el.value

    # ---- adjoint --------------------------------------------------------
    def adjoint_attach(self):
        need = C.c_size_t()
        check(lib().mlbm_adjoint_workspace_bytes(self._h, self.plan.handle, C.byref(need)))
        ws = self.torch.empty(need.value + 256, dtype=self.torch.uint8, device=self.device)
        shift = (-ws.data_ptr()) % 256
        self.adj_workspace = ws
        check(lib().mlbm_adjoint_attach(self._h, self.plan.handle,
                                        C.c_void_p(ws.data_ptr() + shift), need.value))

    def adjoint_seed(self, objective: str = "ke"):
        check(lib().mlbm_adjoint_seed(self._h, {"ke": _lib.OBJ_KE,
                                                "drag_x": _lib.OBJ_DRAG_X}[objective]))

    def adjoint_step(self, ckpt):
        check(lib().mlbm_adjoint_step(self._h, self._ptr(ckpt), ckpt.numel()))

    def adjoint_init(self, rho, u, S=None, want_rho=False, want_S=False):
        """rho, u, S: per-level lists of the tensors given to init.  Returns
        per-level dJ/du (d, n_fluid) [and dJ/drho, dJ/dS]."""
        torch = self.torch
        n = self.plan.n_levels
        arr = C.c_void_p * n
        def ptrs(ts):
            return arr(*[C.c_void_p(t.data_ptr()) if t is not None else None for t in ts])
        du = [torch.empty((self.plan.d, self.plan.info[k]["n_fluid"]), dtype=torch.float64,
                          device=self.device) for k in range(n)]
        dr = [torch.empty(self.plan.info[k]["n_fluid"], dtype=torch.float64, device=self.device)
              for k in range(n)] if want_rho else None
        ns = 6 if self.plan.d == 3 else 3
        dS = [torch.empty((ns, self.plan.info[k]["n_fluid"]), dtype=torch.float64,
                          device=self.device) for k in range(n)] if want_S else None
        for k in range(n):
            nf = self.plan.info[k]["n_fluid"]
            assert rho[k].numel() == nf and u[k].numel() == self.plan.d * nf
            assert S is None or S[k] is None or S[k].numel() == ns * nf
        check(lib().mlbm_adjoint_init(self._h, ptrs(rho), ptrs(u),
                                      ptrs(S) if S is not None else None, ptrs(du),
                                      ptrs(dr) if dr else None, ptrs(dS) if dS else None))
        out = [du]
        if want_rho:
            out.append(dr)
        if want_S:
            out.append(dS)
        return out[0] if len(out) == 1 else tuple(out)

    def adjoint_params(self):
        """(dJ/dtau0, [dJ/domega_L], dJ/du_in (3,))."""
        t = C.c_double()
        w = (C.c_double * self.plan.n_levels)()
        u = (C.c_double * 3)()
        check(lib().mlbm_adjoint_params(self._h, C.byref(t), w, u))
        return t.value, list(w), np.array(list(u))

    def adjoint_lambda(self, k: int):
        out = self.torch.empty((self.plan.q, self.plan.info[k]["n"]), dtype=self.torch.float64,
                               device=self.device)
        check(lib().mlbm_adjoint_get_lambda(self._h, k, self._ptr(out)))
        return out

    def launches_per_step(self) -> int:
        n = C.c_int64()
        check(lib().mlbm_launches_per_step(self._h, C.byref(n)))
        return n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().mlbm_sim_destroy(h)
            except Exception:   # interpreter shutdown: modules already torn down
                pass
            self._h = C.c_void_p()
