"""ctypes binding of libfftdg.so (argument marshalling only).

Every step of the scan runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the stream.  If the shared library is
missing, `load()` raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfftdg.so")

OK, E_INVALID, E_NOVALID, E_NOMEM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
OCC, CAP = 0, 1

PARTIAL_DTYPE = np.dtype([("m", "<f8"), ("s", "<f8"), ("psi_min", "<f8"), ("n_valid", "<i4"),
                          ("n_finite", "<i4"), ("argmin", "<i4"), ("scanned", "<i4")])
RESULT_DTYPE = np.dtype([("dG", "<f8"), ("v_site", "<f8"), ("psi_min", "<f8"), ("n_finite", "<i8"),
                         ("n_samples", "<i8")])


class FFTDGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fftdg error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("n_rec", ctypes.c_int32), ("n_fft", ctypes.c_int32), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("precision", ctypes.c_int32),
                ("clash_mode", ctypes.c_int32), ("ljr_cap", ctypes.c_double), ("occ_f", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("configs_per_chunk", ctypes.c_int32), ("energy_xy_direct", ctypes.c_int32),
                ("snapshots_per_pass", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("clash_stream", ctypes.c_int32)]


def _tuning_dict(t: Tuning) -> dict:
    return {"configs_per_chunk": t.configs_per_chunk, "energy_xy_direct": t.energy_xy_direct,
            "snapshots_per_pass": t.snapshots_per_pass, "use_graph": t.use_graph, "fused": t.fused,
            "clash_stream": t.clash_stream}


class BatchC(ctypes.Structure):
    _fields_ = [("n_lig", ctypes.c_int32), ("atom_off", ctypes.c_void_p), ("conf_off", ctypes.c_void_p),
                ("cfg_off", ctypes.c_void_p), ("q", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("conf_xyz", ctypes.c_void_p), ("cfg_conf", ctypes.c_void_p),
                ("cfg_quat", ctypes.c_void_p), ("cfg_select", ctypes.c_void_p)]


EXPORTS = ["fftdg_version", "fftdg_status_string", "fftdg_create", "fftdg_destroy", "fftdg_last_error",
           "fftdg_set_stream", "fftdg_receptor_grids", "fftdg_set_receptors", "fftdg_scan",
           "fftdg_energy_grid", "fftdg_place", "fftdg_reduce", "fftdg_reduce_static", "fftdg_profile", "fftdg_profile_read",
           "fftdg_get_tuning", "fftdg_set_tuning", "fftdg_autotune", "fftdg_config_features",
           "fftdg_mlp_create", "fftdg_mlp_create_ex", "fftdg_mlp_destroy", "fftdg_mlp_last_error", "fftdg_mlp_num_params",
           "fftdg_mlp_set_params", "fftdg_mlp_get_params", "fftdg_mlp_set_skip", "fftdg_mlp_forward", "fftdg_mlp_grad",
           "fftdg_mlp_train_step", "fftdg_proposal_sample", "fftdg_scan_features", "fftdg_is_plan", "fftdg_sample_poses",
           "fftdg_grids_build", "fftdg_grid_energies", "fftdg_pair_energies"]

N_FEATURES = 18
N_SCAN_FEATURES = 3

KERNEL_NAMES = ["lig_fwd_xy", "zprod", "inv_xy_lse", "merge", "rec_spectra", "reduce", "lig_runs", "clash"]

_lib = None


def load():
    """Load libfftdg.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1708_07045_amd/build.py "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    p, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.fftdg_version.restype = ctypes.c_int
    L.fftdg_status_string.argtypes = [ctypes.c_int]
    L.fftdg_status_string.restype = ctypes.c_char_p
    L.fftdg_create.argtypes = [ctypes.POINTER(p), ctypes.POINTER(GridDesc), ctypes.c_int, p]
    L.fftdg_destroy.argtypes = [p]
    L.fftdg_destroy.restype = None
    L.fftdg_last_error.argtypes = [p]
    L.fftdg_last_error.restype = ctypes.c_char_p
    L.fftdg_set_stream.argtypes = [p, p]
    L.fftdg_receptor_grids.argtypes = [p, i32, p, p, p, p, p, p]
    L.fftdg_set_receptors.argtypes = [p, i32, p, p, p]
    L.fftdg_scan.argtypes = [p, ctypes.POINTER(BatchC), d, p]
    L.fftdg_energy_grid.argtypes = [p, i32, ctypes.POINTER(BatchC), i32, d, p, p, p]
    L.fftdg_place.argtypes = [p, ctypes.POINTER(BatchC), i32, p, p]
    L.fftdg_reduce.argtypes = [p, ctypes.POINTER(BatchC), p, p, d, p, p]
    L.fftdg_reduce_static.argtypes = [p, ctypes.POINTER(BatchC), p, p, d, p, p]
    L.fftdg_profile.argtypes = [p, ctypes.c_int]
    L.fftdg_profile_read.argtypes = [p, i32, p, p, p]
    L.fftdg_get_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
    L.fftdg_set_tuning.argtypes = [p, ctypes.POINTER(Tuning)]
    L.fftdg_autotune.argtypes = [p, ctypes.POINTER(BatchC), d, i32, ctypes.POINTER(Tuning), p]
    L.fftdg_config_features.argtypes = [p, ctypes.POINTER(BatchC), p]
    L.fftdg_mlp_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, p, i32, i32, i32]
    L.fftdg_mlp_create_ex.argtypes = [ctypes.POINTER(p), ctypes.c_int, p, i32, i32, i32, i32]
    L.fftdg_mlp_destroy.argtypes = [p]
    L.fftdg_mlp_destroy.restype = None
    L.fftdg_mlp_last_error.argtypes = [p]
    L.fftdg_mlp_last_error.restype = ctypes.c_char_p
    L.fftdg_mlp_num_params.argtypes = [p]
    L.fftdg_mlp_set_params.argtypes = [p, p, ctypes.c_int64]
    L.fftdg_mlp_get_params.argtypes = [p, p, ctypes.c_int64]
    L.fftdg_mlp_set_skip.argtypes = [p, i32, ctypes.c_float]
    L.fftdg_mlp_forward.argtypes = [p, p, i32, p]
    L.fftdg_mlp_grad.argtypes = [p, p, p, p, p, i32, p, p]
    L.fftdg_mlp_train_step.argtypes = [p, p, p, p, p, i32, ctypes.c_float, p]
    L.fftdg_proposal_sample.argtypes = [p, p, i32, d, d, i32, p, p, p]
    L.fftdg_scan_features.argtypes = [p, ctypes.POINTER(BatchC), p, p, i32, i32]
    L.fftdg_is_plan.argtypes = [p, ctypes.POINTER(BatchC), p, d, d, d, d, p, ctypes.c_int64, p, p, p]
    L.fftdg_sample_poses.argtypes = [p, ctypes.POINTER(BatchC), p, i32, i32, d, i32, p, p, p, p]
    L.fftdg_grids_build.argtypes = [ctypes.c_int, p, ctypes.POINTER(GridDesc), i32, p, p, p, p, p, p]
    L.fftdg_grid_energies.argtypes = [ctypes.c_int, p, ctypes.POINTER(GridDesc), p, i32, i32, p, p, p, p, p]
    L.fftdg_pair_energies.argtypes = [ctypes.c_int, p, i32, p, p, p, p, i32, i32, p, p, p, p, i32, p]
    for name in EXPORTS:
        if name not in ("fftdg_destroy", "fftdg_status_string", "fftdg_last_error", "fftdg_mlp_destroy",
                        "fftdg_mlp_last_error", "fftdg_mlp_num_params"):
            getattr(L, name).restype = ctypes.c_int
    L.fftdg_mlp_num_params.restype = ctypes.c_int64
    _lib = L
    return L


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


class Batch:
    """Host arrays of a batch of ligands and configurations (fftdg_batch)."""

    def __init__(self, ligands: Sequence, select: Optional[np.ndarray] = None):
        n_lig = len(ligands)
        self.n_lig = n_lig
        self.atom_off = np.zeros(n_lig + 1, np.int32)
        self.conf_off = np.zeros(n_lig + 1, np.int32)
        self.cfg_off = np.zeros(n_lig + 1, np.int32)
        for l, L in enumerate(ligands):
            self.atom_off[l + 1] = self.atom_off[l] + L.n_atoms
            self.conf_off[l + 1] = self.conf_off[l] + L.conformers.shape[0]
            self.cfg_off[l + 1] = self.cfg_off[l] + L.n_cfg
        cat = lambda xs, dt: np.ascontiguousarray(np.concatenate(xs), dtype=dt)
        self.q = cat([L.q for L in ligands], np.float64)
        self.sigma = cat([L.sigma for L in ligands], np.float64)
        self.eps = cat([L.eps for L in ligands], np.float64)
        self.conf_xyz = cat([L.conformers.reshape(-1, 3) for L in ligands], np.float64)
        self.cfg_conf = cat([L.cfg_conf for L in ligands], np.int32)
        self.cfg_quat = cat([L.cfg_quat for L in ligands], np.float64)
        self.n_cfg = int(self.cfg_off[-1])
        self.select = self._select_array(select)
        self.c = BatchC(n_lig, _ptr(self.atom_off), _ptr(self.conf_off), _ptr(self.cfg_off), _ptr(self.q),
                        _ptr(self.sigma), _ptr(self.eps), _ptr(self.conf_xyz), _ptr(self.cfg_conf),
                        _ptr(self.cfg_quat), _ptr(self.select))

    def _select_array(self, select):
        """cfg_select: one byte per configuration of the batch (the library
        reads n_cfg of them), or None."""
        if select is None:
            return None
        a = np.ascontiguousarray(select, np.uint8).reshape(-1)
        if a.size != self.n_cfg:
            raise ValueError(f"select has {a.size} entries, the batch {self.n_cfg} configurations")
        return a

    def with_select(self, select: Optional[np.ndarray]) -> "Batch":
        b = object.__new__(Batch)
        b.__dict__.update(self.__dict__)
        b.select = self._select_array(select)
        b.c = BatchC(*[getattr(self.c, f) for f, _ in BatchC._fields_])
        b.c.cfg_select = _ptr(b.select)
        return b


class FFTDG:
    """One library context (one device, one stream)."""

    def __init__(self, n_rec: int, n_fft: int, h: float, origin, precision: str = "f32",
                 clash_mode: str = "occ", ljr_cap: float = 10.0, occ_f: float = 0.5, device: int = 0,
                 stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.precision = precision
        self.clash_mode = clash_mode
        self.n_rec, self.n_fft, self.h = n_rec, n_fft, h
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self.device = torch.device("cuda", device)
        g = GridDesc(n_rec, n_fft, h, (ctypes.c_double * 3)(*[float(x) for x in origin]),
                     F32 if precision == "f32" else F64, OCC if clash_mode == "occ" else CAP,
                     ljr_cap, occ_f)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        h_ = ctypes.c_void_p()
        rc = self.L.fftdg_create(ctypes.byref(h_), ctypes.byref(g), device, ctypes.c_void_p(stream))
        if rc != OK:
            raise FFTDGError(rc, "fftdg_create failed (" + self.L.fftdg_status_string(rc).decode() + ")")
        self.h_ctx = h_
        self.n_snap = 0

    @classmethod
    def from_workload(cls, w, device: int = 0, precision: Optional[str] = None):
        return cls(w.n_rec, w.n_fft, w.h, w.origin, precision or w.precision, w.clash_mode, w.ljr_cap,
                   w.occ_f, device)

    def close(self):
        if getattr(self, "h_ctx", None):
            self.L.fftdg_destroy(self.h_ctx)
            self.h_ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != OK:
            raise FFTDGError(rc, self.L.fftdg_last_error(self.h_ctx).decode())

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(self.L.fftdg_get_tuning(self.h_ctx, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, configs_per_chunk: Optional[int] = None, energy_xy_direct: Optional[int] = None,
                   snapshots_per_pass: Optional[int] = None, use_graph: Optional[int] = None,
                   fused: Optional[int] = None, clash_stream: Optional[int] = None):
        cur = self.get_tuning()
        if configs_per_chunk is not None:
            cur["configs_per_chunk"] = int(configs_per_chunk)
        if energy_xy_direct is not None:
            cur["energy_xy_direct"] = int(energy_xy_direct)
        if snapshots_per_pass is not None:
            cur["snapshots_per_pass"] = int(snapshots_per_pass)
        if use_graph is not None:
            cur["use_graph"] = int(use_graph)
        if fused is not None:
            cur["fused"] = int(fused)
        if clash_stream is not None:
            cur["clash_stream"] = int(clash_stream)
        t = Tuning(cur["configs_per_chunk"], cur["energy_xy_direct"], cur["snapshots_per_pass"],
                   cur["use_graph"], cur["fused"], cur["clash_stream"])
        self._check(self.L.fftdg_set_tuning(self.h_ctx, ctypes.byref(t)))

    def autotune(self, batch: "Batch", T: float, max_cfgs: int = 2048):
        """Pick the fastest schedule on a sample of the batch; returns
        (tuning dict, ms per sampled configuration and snapshot)."""
        t = Tuning()
        ms = ctypes.c_double()
        self._check(self.L.fftdg_autotune(self.h_ctx, ctypes.byref(batch.c), float(T), int(max_cfgs),
                                          ctypes.byref(t), ctypes.byref(ms)))
        return _tuning_dict(t), ms.value

    def set_chunk(self, n: int):
        self.set_tuning(configs_per_chunk=n)

    def profile(self, enable: bool = True):
        self._check(self.L.fftdg_profile(self.h_ctx, 1 if enable else 0))

    def profile_read(self):
        """{kernel name: (ms, launches, algorithmic bytes)} since profile(True)."""
        out = {}
        for k, name in enumerate(KERNEL_NAMES):
            ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
            self._check(self.L.fftdg_profile_read(self.h_ctx, k, ctypes.byref(ms), ctypes.byref(n),
                                                  ctypes.byref(b)))
            out[name] = (ms.value, n.value, b.value)
        return out

    def set_stream(self, stream_handle: int):
        self._check(self.L.fftdg_set_stream(self.h_ctx, ctypes.c_void_p(stream_handle)))

    # ---------------------------------------------------------------- receptor
    def receptor_grids(self, xyz, q, sigma, eps):
        """Eq. 7 / Eq. 10 grids of one receptor snapshot on the GPU."""
        t = self.torch
        dev = lambda a: t.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)
        X, Q, S, E = dev(xyz), dev(q), dev(sigma), dev(eps)
        n = self.n_rec
        grids = t.empty((3, n, n, n), dtype=self.dtype, device=self.device)
        occ = t.empty((n, n, n), dtype=t.uint8, device=self.device) if self.clash_mode == "occ" else None
        self._check(self.L.fftdg_receptor_grids(self.h_ctx, int(X.shape[0]), _ptr(X), _ptr(Q), _ptr(S), _ptr(E),
                                                _ptr(grids), _ptr(occ)))
        self._keep = (X, Q, S, E)
        return grids, occ

    def set_receptors(self, grids, occ=None, weights=None):
        """grids: tensor [n_snap][3][n^3] (or [3][n^3]); occ: [n_snap][n^3] uint8."""
        n_snap = grids.shape[0] if grids.dim() == 5 else 1
        w = None if weights is None else np.ascontiguousarray(weights, np.float64)
        self._check(self.L.fftdg_set_receptors(self.h_ctx, n_snap, _ptr(grids.contiguous()),
                                               _ptr(occ.contiguous()) if occ is not None else None,
                                               _ptr(w)))
        self.n_snap = n_snap

    # ---------------------------------------------------------------- scan
    def alloc_partials(self, batch: Batch):
        return self.torch.empty(self.n_snap * batch.n_cfg * PARTIAL_DTYPE.itemsize, dtype=self.torch.uint8,
                                device=self.device)

    def _partials_ok(self, buf, batch: Batch):
        """The library reads or writes n_snap * n_cfg fftdg_partial records
        through this pointer: a contiguous tensor on this context's device
        holding at least that many bytes."""
        t = self.torch
        need = self.n_snap * batch.n_cfg * PARTIAL_DTYPE.itemsize
        if (not t.is_tensor(buf) or buf.device != self.device or not buf.is_contiguous()
                or buf.numel() * buf.element_size() < need):
            raise ValueError(f"partials: need a contiguous tensor on {self.device} of at least {need} bytes")
        return buf

    def scan(self, batch: Batch, T: float, out=None):
        """Partials [n_snap * n_cfg] (device bytes of fftdg_partial)."""
        if out is None:
            out = self.alloc_partials(batch)
        self._partials_ok(out, batch)
        self._check(self.L.fftdg_scan(self.h_ctx, ctypes.byref(batch.c), float(T), _ptr(out)))
        return out

    @staticmethod
    def partials_numpy(buf, n_snap: int, n_cfg: int) -> np.ndarray:
        a = buf.cpu().numpy().view(PARTIAL_DTYPE)
        return a.reshape(n_snap, n_cfg)

    def energy_grid(self, snap: int, batch: Batch, cfg: int, T: float = 300.0):
        shape = np.zeros(3, np.int32)
        self._check(self.L.fftdg_energy_grid(self.h_ctx, snap, ctypes.byref(batch.c), cfg, float(T), None, None,
                                             _ptr(shape)))
        t = self.torch
        psi = t.zeros(tuple(int(s) for s in shape), dtype=self.dtype, device=self.device)
        clash = t.zeros(tuple(int(s) for s in shape), dtype=t.uint8, device=self.device)
        if psi.numel() > 0:
            self._check(self.L.fftdg_energy_grid(self.h_ctx, snap, ctypes.byref(batch.c), cfg, float(T),
                                                 _ptr(psi), _ptr(clash), _ptr(shape)))
        return psi, clash

    def features(self, batch: Batch) -> np.ndarray:
        """Per-configuration proposal features [n_cfg][N_FEATURES] (host)."""
        f = np.zeros((batch.n_cfg, N_FEATURES), np.float32)
        self._check(self.L.fftdg_config_features(self.h_ctx, ctypes.byref(batch.c), _ptr(f)))
        return f

    def place(self, batch: Batch, cfg: int):
        l = int(np.searchsorted(batch.cfg_off, cfg, side="right") - 1)
        na = int(batch.atom_off[l + 1] - batch.atom_off[l])
        U = np.zeros((na, 3), np.int32)
        box = np.zeros(3, np.int32)
        self._check(self.L.fftdg_place(self.h_ctx, ctypes.byref(batch.c), cfg, _ptr(U), _ptr(box)))
        return U, box

    def boxes(self, batch: Batch) -> np.ndarray:
        """Box extents (x, y, z) of every configuration of the batch as the
        scan places it, [n_cfg][3] (one fftdg_place call each)."""
        out = np.zeros((batch.n_cfg, 3), np.int32)
        na_max = int(np.max(np.diff(batch.atom_off)))
        U = np.zeros((na_max, 3), np.int32)
        for c in range(batch.n_cfg):
            self._check(self.L.fftdg_place(self.h_ctx, ctypes.byref(batch.c), c, _ptr(U), _ptr(out[c])))
        return out

    def scan_features(self, batch: Batch, partials, feat, col0: int):
        """Write the N_SCAN_FEATURES descriptors of this context's scan into
        columns col0.. of the device float matrix feat [n_cfg][ld]."""
        t = self.torch
        assert feat.dtype == t.float32 and feat.dim() == 2 and feat.is_contiguous()
        assert feat.shape[0] == batch.n_cfg
        self._partials_ok(partials, batch)
        self._check(self.L.fftdg_scan_features(self.h_ctx, ctypes.byref(batch.c), _ptr(partials), _ptr(feat),
                                               int(feat.shape[1]), int(col0)))
        return feat

    def is_plan(self, batch: Batch, yhat, top_frac: float, draw_frac: float, alpha: float, tau: float,
                uniforms):
        """Stratified importance-sampling plan (see is_plan)."""
        return is_plan(batch, yhat, top_frac, draw_frac, alpha, tau, uniforms, self)

    def sample_poses(self, batch: Batch, partials, lig: int, snap: int, T: float, uniforms):
        """Sampling importance resampling of len(uniforms)//2 poses:
        (configuration index [K], translation (tx, ty, tz) [K][3], Psi [K])."""
        u = np.ascontiguousarray(uniforms, np.float64)
        K = u.size // 2
        cfg = np.zeros(K, np.int32)
        t = np.zeros((K, 3), np.int32)
        psi = np.zeros(K, np.float64)
        self._partials_ok(partials, batch)
        self._check(self.L.fftdg_sample_poses(self.h_ctx, ctypes.byref(batch.c), _ptr(partials), int(lig), int(snap),
                                              float(T), K, _ptr(u), _ptr(cfg), _ptr(t), _ptr(psi)))
        return cfg, t, psi

    def reduce(self, batch: Batch, partials, T: float, cfg_weight=None):
        return self._reduce(self.L.fftdg_reduce, batch, partials, T, cfg_weight)

    def reduce_static(self, batch: Batch, partials, T: float, cfg_weight=None):
        """fftdg_reduce_static: the same results with the library's static
        device scratch (no device allocation in the call; cfg_weight, if
        given, should already be a float64 device tensor)."""
        return self._reduce(self.L.fftdg_reduce_static, batch, partials, T, cfg_weight)

    def _reduce(self, fn, batch, partials, T, cfg_weight):
        self._partials_ok(partials, batch)
        B = np.zeros((batch.n_lig, self.n_snap), np.float64)
        res = np.zeros(batch.n_lig, RESULT_DTYPE)
        w = cfg_weight
        if cfg_weight is not None:
            if self.torch.is_tensor(cfg_weight) and cfg_weight.is_cuda:
                if (cfg_weight.dtype != self.torch.float64 or not cfg_weight.is_contiguous()
                        or cfg_weight.numel() != batch.n_cfg):
                    raise ValueError("cfg_weight: need a contiguous float64 device tensor of n_cfg entries")
            else:
                w = np.ascontiguousarray(cfg_weight, np.float64).reshape(-1)
                if w.size != batch.n_cfg:
                    raise ValueError(f"cfg_weight: {w.size} entries for {batch.n_cfg} configurations")
                w = self.torch.as_tensor(w, device=self.device)
        self._check(fn(self.h_ctx, ctypes.byref(batch.c), _ptr(partials), _ptr(w), float(T), _ptr(B), _ptr(res)))
        return B, res


class GridTools:
    """Grids and pose energies without an FFT context (fftdg_grids_build,
    fftdg_grid_energies, fftdg_pair_energies) on one device and stream."""

    def __init__(self, n_rec: int, h: float, origin, precision: str = "f64", clash_mode: str = "occ",
                 ljr_cap: float = 10.0, occ_f: float = 0.5, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.device = torch.device("cuda", device)
        self.dev_index = device
        self.n_rec, self.h = n_rec, h
        self.precision, self.clash_mode = precision, clash_mode
        self.g = GridDesc(n_rec, 0, h, (ctypes.c_double * 3)(*[float(x) for x in origin]),
                          F32 if precision == "f32" else F64, OCC if clash_mode == "occ" else CAP, ljr_cap, occ_f)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream

    def _d(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, np.float64), device=self.device)

    @staticmethod
    def _rc(rc, what):
        if rc != OK:
            raise FFTDGError(rc, what + " failed (" + load().fftdg_status_string(rc).decode() + ")")

    def build(self, xyz, q, sigma, eps):
        t = self.torch
        n = self.n_rec
        grids = t.empty((3, n, n, n), dtype=t.float32 if self.precision == "f32" else t.float64, device=self.device)
        occ = t.empty((n, n, n), dtype=t.uint8, device=self.device) if self.clash_mode == "occ" else None
        X, Q, S, E = self._d(xyz), self._d(q), self._d(sigma), self._d(eps)
        self._rc(self.L.fftdg_grids_build(self.dev_index, ctypes.c_void_p(self.stream), ctypes.byref(self.g),
                                          int(X.shape[0]), _ptr(X), _ptr(Q), _ptr(S), _ptr(E), _ptr(grids),
                                          _ptr(occ)), "fftdg_grids_build")
        t.cuda.synchronize(self.device)
        return grids, occ

    def grid_energies(self, grids, poses, q, sigma, eps):
        """poses [n_poses][n_atoms][3] (Angstrom) -> [n_poses][3] (ELE, LJr, LJa)."""
        P = self._d(poses)
        Q, S, E = self._d(q), self._d(sigma), self._d(eps)
        out = self.torch.empty((P.shape[0], 3), dtype=self.torch.float64, device=self.device)
        self._rc(self.L.fftdg_grid_energies(self.dev_index, ctypes.c_void_p(self.stream), ctypes.byref(self.g),
                                            _ptr(grids), int(P.shape[0]), int(P.shape[1]), _ptr(Q), _ptr(S), _ptr(E),
                                            _ptr(P), _ptr(out)), "fftdg_grid_energies")
        return out.cpu().numpy()

    def pair_energies(self, rxyz, rq, rsigma, reps, poses, q, sigma, eps, exclusion: bool = True):
        R, RQ, RS, RE = self._d(rxyz), self._d(rq), self._d(rsigma), self._d(reps)
        P = self._d(poses)
        Q, S, E = self._d(q), self._d(sigma), self._d(eps)
        out = self.torch.empty((P.shape[0], 3), dtype=self.torch.float64, device=self.device)
        self._rc(self.L.fftdg_pair_energies(self.dev_index, ctypes.c_void_p(self.stream), int(R.shape[0]), _ptr(R),
                                            _ptr(RQ), _ptr(RS), _ptr(RE), int(P.shape[0]), int(P.shape[1]), _ptr(Q),
                                            _ptr(S), _ptr(E), _ptr(P), 1 if exclusion else 0, _ptr(out)),
                 "fftdg_pair_energies")
        return out.cpu().numpy()


def is_plan(batch: Batch, yhat, top_frac: float, draw_frac: float, alpha: float, tau: float, uniforms,
            ctx: Optional["FFTDG"] = None):
    """fftdg_is_plan (host only): (select uint8 [n_cfg], weight float64
    [n_cfg], number of configurations selected)."""
    L = load()
    y = yhat.detach().float().cpu().numpy() if hasattr(yhat, "detach") else np.asarray(yhat)
    y = np.ascontiguousarray(y, np.float32)
    u = np.ascontiguousarray(uniforms, np.float64)
    sel = np.zeros(batch.n_cfg, np.uint8)
    wt = np.zeros(batch.n_cfg, np.float64)
    n = ctypes.c_int64()
    h = ctx.h_ctx if ctx is not None else None
    rc = L.fftdg_is_plan(h, ctypes.byref(batch.c), _ptr(y), float(top_frac), float(draw_frac), float(alpha),
                         float(tau), _ptr(u), int(u.size), _ptr(sel), _ptr(wt), ctypes.byref(n))
    if rc != OK:
        msg = L.fftdg_last_error(h).decode() if h else L.fftdg_status_string(rc).decode()
        raise FFTDGError(rc, "fftdg_is_plan: " + msg)
    return sel, wt, int(n.value)


class Network:
    """The proposal network of the library (fftdg_mlp); fp32: FP32 operands
    and activations instead of BF16 (fftdg_mlp_create_ex)."""

    def __init__(self, n_in: int = N_FEATURES, width: int = 256, max_batch: int = 4096, device: int = 0,
                 stream=None, fp32: bool = False):
        import torch
        self.torch = torch
        self.L = load()
        self.n_in, self.width, self.max_batch = n_in, width, max_batch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        rc = self.L.fftdg_mlp_create_ex(ctypes.byref(h), device, ctypes.c_void_p(stream), n_in, width, max_batch,
                                        1 if fp32 else 0)
        if rc != OK:
            raise FFTDGError(rc, "fftdg_mlp_create_ex failed (" + self.L.fftdg_status_string(rc).decode() + ")")
        self.h = h
        self.n_params = int(self.L.fftdg_mlp_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            self.L.fftdg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise FFTDGError(rc, self.L.fftdg_mlp_last_error(self.h).decode())

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, np.float32)
        self._check(self.L.fftdg_mlp_set_params(self.h, _ptr(p), p.size))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, np.float32)
        self._check(self.L.fftdg_mlp_get_params(self.h, _ptr(p), p.size))
        return p

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(self.device, dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), device=self.device).to(dtype).contiguous()

    def set_skip(self, col: int, scale: float = 1.0):
        """Output net(x) + scale * x[col] (col = -1: none)."""
        self._check(self.L.fftdg_mlp_set_skip(self.h, int(col), float(scale)))

    def forward(self, X):
        t = self.torch
        x = self._dev(X, t.float32)
        y = t.empty(x.shape[0], dtype=t.float32, device=self.device)
        self._check(self.L.fftdg_mlp_forward(self.h, _ptr(x), int(x.shape[0]), _ptr(y)))
        return y

    def grad(self, X, T, W, idx=None):
        t = self.torch
        x, tt, ww = self._dev(X, t.float32), self._dev(T, t.float32), self._dev(W, t.float32)
        ii = None if idx is None else self._dev(idx, t.int32)
        B = int(x.shape[0] if ii is None else ii.shape[0])
        g = t.zeros(self.n_params, dtype=t.float32, device=self.device)
        loss = ctypes.c_float()
        self._check(self.L.fftdg_mlp_grad(self.h, _ptr(x), _ptr(tt), _ptr(ww), _ptr(ii), B, _ptr(g),
                                          ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, x, t_, w, idx, lr: float, want_loss: bool = False):
        """x, t_, w, idx: device tensors (float32, float32, float32, int32)."""
        loss = ctypes.c_float()
        self._check(self.L.fftdg_mlp_train_step(self.h, _ptr(x), _ptr(t_), _ptr(w), _ptr(idx), int(idx.shape[0]),
                                                float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def sample(self, yhat, alpha: float, tau: float, uniforms):
        """Mixture proposal q [P] (float64) and len(uniforms) draws (int32)."""
        t = self.torch
        y = self._dev(yhat, t.float32)
        u = self._dev(uniforms, t.float64)
        P, K = int(y.shape[0]), int(u.shape[0])
        idx = t.empty(K, dtype=t.int32, device=self.device)
        q = t.empty(P, dtype=t.float64, device=self.device)
        self._check(self.L.fftdg_proposal_sample(self.h, _ptr(y), P, float(alpha), float(tau), K, _ptr(u),
                                                 _ptr(idx), _ptr(q)))
        return q, idx
