"""paper_2402_13861_amd -- hierarchical iso-surface extraction on ReLU INRs
for AMD MI355X (gfx950).

A thin Python binding over the C ABI of ``libisx.so`` (``include/isx.h``):
arguments are marshalled here, every step of the computation runs in the
library's HIP kernels.  Device buffers are torch CUDA (HIP) tensors; torch
provides device memory and streams only.

Method: Li & Shen, arXiv 2402.13861 -- range analysis by affine arithmetic
(Sec. III) and uncertainty propagation (Sec. IV), hierarchical extraction
(Alg. 1), marching cubes on active leaves (Sec. IV-D).
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (AA, RAUA, RAFIXED, RELU, SINE, ELU, BF16, BF16_VARIANT, FP32, FP64, HIDDEN_KERNEL, KEEP_LEVELS, PROFILE, SCRATCH_BYTES, UP,
                   UP_FORM, LIN_PRECISION, AA_MARGIN, BATCH_WORKERS, VERBOSE, CANCEL_CHECK, AUTOTUNE,
                   BF16_READOFF, RECHECK_CASCADE, DENSE_FROM_LEVEL, RECHECK_SPLIT)

# columns of isx_distribution_kl's report (isx_dist_field order)
DIST_FIELDS = ("mc_mean", "mc_std", "lo", "hi", "up_mu", "up_sigma", "raua_mu", "raua_sigma", "fit_mu", "fit_sigma",
               "kl_up", "kl_raua", "kl_fit")
KERNEL_KINDS = ("hidden_fp32", "hidden_bf16", "hidden_simt_fp32", "hidden_fp64", "dense", "output",
                "hidden_cov_bf16", "linearize")

__all__ = ["Context", "Mesh", "IsxError", "AA", "UP", "RAUA", "RAFIXED", "RELU", "SINE", "ELU", "FP32", "BF16", "FP64", "KEEP_LEVELS", "HIDDEN_KERNEL",
           "PROFILE", "SCRATCH_BYTES", "VERBOSE", "BF16_VARIANT", "mc_case_table"]


class IsxError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to libisx must be contiguous")
    return t.data_ptr()


def _check_dev(t, dtype, name, shape_tail=None):
    import torch

    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    del torch


def mc_case_table():
    """The library's marching-cubes table: (count[256] uint8, edges[256,15] int8)."""
    cnt = np.zeros(256, dtype=np.uint8)
    edg = np.zeros((256, 15), dtype=np.int8)
    _lib.lib().isx_mc_case_table(cnt.ctypes.data, edg.ctypes.data)
    return cnt, edg


class Context:
    """One library context on a HIP device and stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self._L = _lib.lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        p = C.c_void_p()
        st = self._L.isx_create(device, C.c_void_p(handle), C.byref(p))
        if st != 0:
            raise IsxError(st, self._L.isx_last_error(None).decode())
        self._h = p
        self.device = device

    def _chk(self, st):
        if st != 0:
            raise IsxError(st, self._L.isx_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.isx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- weights / configuration
    def load_mlp(self, Ws: Sequence[np.ndarray], bs: Sequence[np.ndarray]) -> int:
        Ws = [np.ascontiguousarray(W, dtype=np.float32) for W in Ws]
        bs = [np.ascontiguousarray(b, dtype=np.float32) for b in bs]
        widths = [Ws[0].shape[1]] + [W.shape[0] for W in Ws]
        n = len(Ws)
        w_arr = (C.c_int32 * (n + 1))(*widths)
        Wp = (C.c_void_p * n)(*[W.ctypes.data for W in Ws])
        bp = (C.c_void_p * n)(*[b.ctypes.data for b in bs])
        out = C.c_int32()
        self._chk(self._L.isx_load_mlp(self._h, n, w_arr, Wp, bp, C.byref(out)))
        return out.value

    def load_weights(self, mlp) -> int:
        """Load a ``workloads.MLPWeights``-like object (``Ws``, ``bs``)."""
        return self.load_mlp(mlp.Ws, mlp.bs)

    def unload_mlp(self, mlp_id: int):
        self._chk(self._L.isx_unload_mlp(self._h, mlp_id))

    def set_activation(self, mlp_id: int, act: int):
        """Hidden activation of a loaded MLP: RELU (default), SINE or ELU."""
        self._chk(self._L.isx_set_activation(self._h, mlp_id, int(act)))

    def set_domain(self, mlp_id: int, lo, hi):
        lo = (C.c_float * 3)(*map(float, lo))
        hi = (C.c_float * 3)(*map(float, hi))
        self._chk(self._L.isx_set_domain(self._h, mlp_id, lo, hi))

    def set_isovalues(self, mlp_id: int, isos):
        isos = [float(x) for x in np.atleast_1d(isos)]
        arr = (C.c_float * max(1, len(isos)))(*isos)
        self._chk(self._L.isx_set_isovalues(self._h, mlp_id, len(isos), arr))

    def set_option(self, option: int, value: int):
        self._chk(self._L.isx_set_option(self._h, option, int(value)))

    def profile(self, reset: bool = True):
        """Kernel statistics per kind (ISX_PROFILE on): {kind name: dict of
        launches, ms, flops, bytes}; reset clears them afterwards."""
        out = {}
        for kind, name in enumerate(KERNEL_KINDS):
            n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            self._chk(self._L.isx_get_profile(self._h, kind, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by), 0))
            out[name] = dict(launches=n.value, ms=ms.value, flops=fl.value, bytes=by.value)
        if reset:
            self._chk(self._L.isx_get_profile(self._h, 0, None, None, None, None, 1))
        return out

    # -- batched calls on device tensors (asynchronous on the context stream)
    def propagate(self, mlp_id: int, method: int, precision: int, centres, halves, out, out64=None):
        import torch

        _check_dev(centres, torch.float32, "centres", (3,))
        _check_dev(halves, torch.float32, "halves", (3,))
        _check_dev(out, torch.float32, "out", (2,))
        _check_dev(out64, torch.float64, "out64", (2,))
        n = centres.shape[0]
        if halves.shape[0] != n or out.shape[0] != n or (out64 is not None and out64.shape[0] != n):
            raise ValueError("centres, halves and out must have the same length")
        self._chk(self._L.isx_propagate(self._h, mlp_id, method, precision, n, _ptr(centres), _ptr(halves),
                                        _ptr(out), _ptr(out64)))

    def classify_compact(self, mlp_id: int, k: float, out, parent_mask=None):
        """Returns (active_idx, active_mask, n_active) device tensors; the
        first n_active entries are valid."""
        import torch

        _check_dev(out, torch.float32, "out", (2,))
        n = out.shape[0]
        if parent_mask is not None:
            _check_dev(parent_mask, torch.int32, "parent_mask")
        idx = torch.empty(max(n, 1), dtype=torch.int32, device=out.device)
        msk = torch.empty(max(n, 1), dtype=torch.int32, device=out.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=out.device)
        self._chk(self._L.isx_classify_compact(self._h, mlp_id, float(k), n, _ptr(out), _ptr(parent_mask),
                                               _ptr(idx), _ptr(msk), _ptr(cnt)))
        return idx, msk, cnt

    def classify_compact_noalloc(self, mlp_id: int, k: float, out, parent_mask, idx, msk, cnt):
        """isx_classify_compact_noalloc into caller-allocated device tensors
        idx, msk (int32 [>= n]) and cnt (int64 [1]); allocates nothing."""
        n = out.shape[0]
        self._chk(self._L.isx_classify_compact_noalloc(self._h, mlp_id, float(k), n, _ptr(out), _ptr(parent_mask),
                                                       _ptr(idx), _ptr(msk), _ptr(cnt)))

    # -- learned surrogate
    def surrogate_load(self, Ws, bs) -> int:
        Ws = [np.ascontiguousarray(W, dtype=np.float32) for W in Ws]
        bs = [np.ascontiguousarray(b, dtype=np.float32) for b in bs]
        widths = [Ws[0].shape[1]] + [W.shape[0] for W in Ws]
        n = len(Ws)
        out = C.c_int32()
        self._chk(self._L.isx_surrogate_load(self._h, n, (C.c_int32 * (n + 1))(*widths),
                                             (C.c_void_p * n)(*[W.ctypes.data for W in Ws]),
                                             (C.c_void_p * n)(*[b.ctypes.data for b in bs]), C.byref(out)))
        self._sur_shapes = getattr(self, "_sur_shapes", {})
        self._sur_shapes[out.value] = [W.shape for W in Ws]
        return out.value

    def surrogate_weights(self, sid: int):
        shapes = self._sur_shapes[sid]
        Ws = [np.zeros(s, dtype=np.float32) for s in shapes]
        bs = [np.zeros(s[0], dtype=np.float32) for s in shapes]
        n = len(Ws)
        self._chk(self._L.isx_surrogate_get(self._h, sid, (C.c_void_p * n)(*[W.ctypes.data for W in Ws]),
                                            (C.c_void_p * n)(*[b.ctypes.data for b in bs])))
        return Ws, bs

    def surrogate_set_norm(self, sid: int, mu_bar: float, scale: float, size_a: float, size_b: float):
        self._chk(self._L.isx_surrogate_set_norm(self._h, sid, float(mu_bar), float(scale), float(size_a),
                                                 float(size_b)))

    def surrogate_set_base(self, sid: int, mlp_id: int, s_floor: float = 0.0):
        """Outputs become corrections to ``mlp_id``'s centre linearisation
        (mlp_id = -1: standardised targets)."""
        self._chk(self._L.isx_surrogate_set_base(self._h, sid, int(mlp_id), float(s_floor)))

    def surrogate_train(self, sid: int, centres, halves, targets, steps: int, batch: int, lr: float,
                        first_row: int = 0, loss=None):
        import torch

        _check_dev(centres, torch.float32, "centres", (3,))
        _check_dev(halves, torch.float32, "halves", (3,))
        _check_dev(targets, torch.float32, "targets", (2,))
        _check_dev(loss, torch.float32, "loss")
        self._chk(self._L.isx_surrogate_train(self._h, sid, centres.shape[0], _ptr(centres), _ptr(halves),
                                              _ptr(targets), int(first_row), int(steps), int(batch), float(lr),
                                              _ptr(loss)))

    def surrogate_grad(self, sid: int, centres, halves, targets, batch: int, first_row: int = 0):
        shapes = self._sur_shapes[sid]
        gW = [np.zeros(s, dtype=np.float32) for s in shapes]
        gb = [np.zeros(s[0], dtype=np.float32) for s in shapes]
        n = len(gW)
        loss = C.c_float()
        self._chk(self._L.isx_surrogate_grad(self._h, sid, centres.shape[0], _ptr(centres), _ptr(halves),
                                             _ptr(targets), int(first_row), int(batch),
                                             (C.c_void_p * n)(*[g.ctypes.data for g in gW]),
                                             (C.c_void_p * n)(*[g.ctypes.data for g in gb]), C.byref(loss)))
        return gW, gb, loss.value

    def surrogate_predict(self, sid: int, centres, halves, out):
        import torch

        _check_dev(out, torch.float32, "out", (2,))
        self._chk(self._L.isx_surrogate_predict(self._h, sid, centres.shape[0], _ptr(centres), _ptr(halves),
                                                _ptr(out)))

    def surrogate_attach(self, mlp_id: int, sid: int, err_mu, err_logsig, z=2.0, accept_leaves: bool = False,
                         z_accept=None):
        """z: band for pruning; z_accept: band for accepting (default z);
        each a scalar or one value per level."""
        err_mu = [float(x) for x in err_mu]
        err_ls = [float(x) for x in err_logsig]
        n = len(err_mu)

        def per_level(v):
            v = [float(v)] * n if np.isscalar(v) else [float(x) for x in v]
            if len(v) != n:
                raise ValueError("band arrays need one value per level")
            return v

        zp = per_level(z)
        za = per_level(z if z_accept is None else z_accept)
        self._chk(self._L.isx_surrogate_attach(self._h, mlp_id, sid, n, (C.c_float * n)(*err_mu),
                                               (C.c_float * n)(*err_ls), (C.c_float * n)(*zp),
                                               (C.c_float * n)(*za), int(bool(accept_leaves))))

    def surrogate_partition(self, mlp_id: int, pred, unit, k: float, level: int, leaf: bool, parent_mask):
        """isx_surrogate_partition on device tensors: pred float32 [n, 2],
        unit float32 [n] or None, parent_mask int32 [n]; returns (mask,
        fallback) int32 device tensors."""
        import torch

        _check_dev(pred, torch.float32, "pred", (2,))
        n = pred.shape[0]
        mask = torch.empty(max(n, 1), dtype=torch.int32, device=pred.device)
        fb = torch.empty(max(n, 1), dtype=torch.int32, device=pred.device)
        self._chk(self._L.isx_surrogate_partition(self._h, mlp_id, n, _ptr(pred), _ptr(unit), float(k), int(level),
                                                  int(bool(leaf)), _ptr(parent_mask), _ptr(mask), _ptr(fb)))
        return mask[:n], fb[:n]

    def propagate_segments(self, mlp_id: int, method: int, precision: int, centres, halfvec, out, out64=None):
        """isx_propagate_segments on device tensors: centres and half-vectors
        float32 [n, 3], out float32 [n, 2] (and float64 out64 with FP64)."""
        import torch

        _check_dev(centres, torch.float32, "centres", (3,))
        _check_dev(halfvec, torch.float32, "halfvec", (3,))
        _check_dev(out, torch.float32, "out", (2,))
        _check_dev(out64, torch.float64, "out64", (2,))
        n = centres.shape[0]
        if halfvec.shape[0] != n or out.shape[0] != n or (out64 is not None and out64.shape[0] != n):
            raise ValueError("centres, halfvec and out must have the same length")
        self._chk(self._L.isx_propagate_segments(self._h, mlp_id, method, precision, n, _ptr(centres), _ptr(halfvec),
                                                 _ptr(out), _ptr(out64)))

    def raycast(self, mlp_id: int, origins, dirs, tnear, tfar, method: int = UP, precision: int = FP32,
                k: float = 3.0, iso: float = 0.0, step0: float = 1.0 / 16, step_min: float = 1.0 / 1024,
                step_max: float = 0.5, max_iter: int = 1000):
        """isx_raycast on device tensors origins/dirs float32 [n, 3], tnear/tfar
        float32 [n]; returns (t_hit float32 [n] with NaN for no hit, steps
        int32 [n], segments bounded, steps of the slowest ray)."""
        import torch

        _check_dev(origins, torch.float32, "origins", (3,))
        _check_dev(dirs, torch.float32, "dirs", (3,))
        n = origins.shape[0]
        for name, t in (("dirs", dirs), ("tnear", tnear), ("tfar", tfar)):
            if t.shape[0] != n:
                raise ValueError(f"{name} must have one row per ray")
        thit = torch.empty(max(n, 1), dtype=torch.float32, device=origins.device)
        iters = torch.empty(max(n, 1), dtype=torch.int32, device=origins.device)
        p = _lib.RayParams(method, precision, float(k), float(iso), float(step0), float(step_min), float(step_max),
                           int(max_iter))
        stats = (C.c_int64 * 2)()
        self._chk(self._L.isx_raycast(self._h, mlp_id, C.byref(p), n, _ptr(origins), _ptr(dirs), _ptr(tnear),
                                      _ptr(tfar), _ptr(thit), _ptr(iters), stats))
        return thit[:n], iters[:n], int(stats[0]), int(stats[1])

    def distribution_kl(self, mlp_id: int, centres, halves, n_samples: int = 1_000_000, n_bins: int = 100,
                        n_fit: int = 100, seed: int = 0, with_hist: bool = False):
        """isx_distribution_kl on device tensors centres/halves float32 [n, 3]:
        returns a float64 [n, 13] tensor (columns DIST_FIELDS) and, with
        with_hist, the int32 [n, n_bins] bin counts."""
        import torch

        _check_dev(centres, torch.float32, "centres", (3,))
        _check_dev(halves, torch.float32, "halves", (3,))
        n = centres.shape[0]
        if halves.shape[0] != n:
            raise ValueError("centres and halves must have the same length")
        out = torch.full((max(n, 1), len(DIST_FIELDS)), float("nan"), dtype=torch.float64, device=centres.device)
        hist = torch.zeros((max(n, 1), n_bins), dtype=torch.int32, device=centres.device) if with_hist else None
        self._chk(self._L.isx_distribution_kl(self._h, mlp_id, n, _ptr(centres), _ptr(halves), int(n_samples),
                                              int(n_bins), int(n_fit), int(seed) & ((1 << 64) - 1), _ptr(out),
                                              _ptr(hist)))
        return (out[:n], hist[:n]) if with_hist else out[:n]

    @staticmethod
    def _calibration(cal):
        n = cal.n_levels
        return dict(n_levels=n, n_cells=list(cal.n_cells[:n]), kept=list(cal.kept[:n]), err_mu=list(cal.err_mu[:n]),
                    err_logsig=list(cal.err_logsig[:n]), z=list(cal.z[:n]), z_accept=list(cal.z_accept[:n]),
                    z_global=cal.z_global, z_accept_global=cal.z_accept_global, holdout_miss=cal.holdout_miss,
                    holdout_false_accept=cal.holdout_false_accept)

    def surrogate_sample_cells(self, mlp_id: int, visited, n: int, level_lo: int, level_hi: int, seed: int = 0):
        """isx_surrogate_sample_cells: (centres, halves, levels) device
        tensors of n training cells; visited is a Mesh made with KEEP_LEVELS
        (or None)."""
        import torch

        dev = torch.device("cuda", self.device)
        c = torch.empty((n, 3), dtype=torch.float32, device=dev)
        h = torch.empty((n, 3), dtype=torch.float32, device=dev)
        lv = torch.empty(n, dtype=torch.int32, device=dev)
        self._chk(self._L.isx_surrogate_sample_cells(self._h, mlp_id, visited._h if visited is not None else None, n,
                                                     level_lo, level_hi, int(seed), _ptr(c), _ptr(h), _ptr(lv)))
        return c, h, lv

    def surrogate_calibrate(self, sid: int, mlp_id: int, centres, halves, targets, levels, n_levels: int, k: float,
                            miss_target: float = 1e-4, accept_target: float = 1e-3, min_level_kept: int = 20000,
                            accept_leaves: bool = False):
        """isx_surrogate_calibrate on held-out device tensors; attaches the
        surrogate and returns its calibration as a dict."""
        cal = _lib.SurrogateCalibration()
        self._chk(self._L.isx_surrogate_calibrate(self._h, sid, mlp_id, centres.shape[0], _ptr(centres), _ptr(halves),
                                                  _ptr(targets), _ptr(levels), n_levels, float(k), float(miss_target),
                                                  float(accept_target), int(min_level_kept), int(bool(accept_leaves)),
                                                  C.byref(cal)))
        return self._calibration(cal)

    def surrogate_fit(self, mlp_id: int, visited=None, *, n_pairs: int, n_holdout: int, steps: int, batch: int,
                      lr: float, seed: int, depth: int, mu_bar: float, scale: float, k: float, use_base: bool,
                      accept_leaves: bool, miss_target: float = 1e-4, accept_target: float = 1e-3,
                      min_level_kept: int = 20000, hidden_width: int = 128, hidden_layers: int = 3):
        """isx_surrogate_fit: returns (surrogate id, calibration dict, losses
        per step as a numpy array)."""
        p = _lib.SurrogateFitParams(n_pairs=n_pairs, n_holdout=n_holdout, steps=steps, batch=batch, lr=lr,
                                    seed=seed, depth=depth, hidden_width=hidden_width, hidden_layers=hidden_layers,
                                    use_base=int(bool(use_base)), mu_bar=mu_bar, scale=scale, k=k,
                                    miss_target=miss_target, accept_target=accept_target,
                                    min_level_kept=min_level_kept, accept_leaves=int(bool(accept_leaves)))
        sid = C.c_int32()
        cal = _lib.SurrogateCalibration()
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        self._chk(self._L.isx_surrogate_fit(self._h, mlp_id, visited._h if visited is not None else None, C.byref(p),
                                            C.byref(sid), C.byref(cal), losses.ctypes.data))
        widths = [4] + [hidden_width] * hidden_layers + [2]
        self._sur_shapes = getattr(self, "_sur_shapes", {})
        self._sur_shapes[sid.value] = [(o, i) for i, o in zip(widths[:-1], widths[1:])]
        return sid.value, self._calibration(cal), losses[:steps]

    def surrogate_free(self, sid: int):
        self._chk(self._L.isx_surrogate_free(self._h, sid))

    def surrogate_save(self, sid: int, path: str):
        """Write surrogate sid (weights, normalisation, base flag) to a file."""
        self._chk(self._L.isx_surrogate_save_file(self._h, sid, str(path).encode()))

    def surrogate_load_file(self, path: str, base_mlp: int = -1) -> int:
        """Read a file written by surrogate_save; base_mlp is the MLP whose
        linearisation a base-mode surrogate corrects (-1 for none)."""
        out = C.c_int32()
        self._chk(self._L.isx_surrogate_load_file(self._h, str(path).encode(), int(base_mlp), C.byref(out)))
        sid = out.value
        # shapes for surrogate_weights: read back from the file header
        with open(path, "rb") as f:
            f.read(8)
            L = int(np.frombuffer(f.read(4), dtype=np.int32)[0])
            w = np.frombuffer(f.read(4 * (L + 1)), dtype=np.int32)
        self._sur_shapes = getattr(self, "_sur_shapes", {})
        self._sur_shapes[sid] = [(int(w[l + 1]), int(w[l])) for l in range(L)]
        return sid

    def eval_points(self, mlp_id: int, precision: int, pts, vals):
        import torch

        _check_dev(pts, torch.float32, "pts", (3,))
        _check_dev(vals, torch.float32, "vals")
        self._chk(self._L.isx_eval_points(self._h, mlp_id, precision, pts.shape[0], _ptr(pts), _ptr(vals)))

    def linearize(self, mlp_id: int, centres, halves, out):
        """(f(c), |J(c) diag(h)| / sqrt 3) per cell into ``out [n, 2]``."""
        import torch

        _check_dev(centres, torch.float32, "centres", (3,))
        _check_dev(halves, torch.float32, "halves", (3,))
        _check_dev(out, torch.float32, "out", (2,))
        n = centres.shape[0]
        if halves.shape[0] != n or out.shape[0] != n:
            raise ValueError("centres, halves and out must have the same length")
        self._chk(self._L.isx_linearize(self._h, mlp_id, n, _ptr(centres), _ptr(halves), _ptr(out)))

    # -- full extraction (synchronous)
    def extract(self, mlp_id: int, method: int = UP, precision: int = FP32, k: float = 3.0, max_depth: int = 6,
                fp64_band: float = 0.0, max_cells: int = 0, chunk_cells: int = 0,
                use_surrogate: bool = False, kd_tree: bool = False, fp64_band_rel: float = 0.0) -> "Mesh":
        """isx_extract; kd_tree selects Alg. 1's binary k-d tree (node depth
        3 max_depth) instead of the octree."""
        p = _lib.Params(method, precision, float(k), int(max_depth), float(fp64_band), int(max_cells),
                        int(chunk_cells), int(bool(use_surrogate)), int(bool(kd_tree)), float(fp64_band_rel))
        h = C.c_void_p()
        self._chk(self._L.isx_extract(self._h, mlp_id, C.byref(p), C.byref(h)))
        return Mesh(self._L, h)

    def extract_dense(self, mlp_id: int, max_depth: int, precision: int = FP32) -> "Mesh":
        """isx_extract_dense: the INR at every corner of the (2^D)^3 grid and
        marching cubes on every cell (the dense baseline)."""
        h = C.c_void_p()
        self._chk(self._L.isx_extract_dense(self._h, int(mlp_id), int(max_depth), int(precision), C.byref(h)))
        return Mesh(self._L, h)

    def extract_batch(self, mlp_ids, method: int = UP, precision: int = FP32, k: float = 3.0, max_depth: int = 6,
                      fp64_band: float = 0.0, max_cells: int = 0, chunk_cells: int = 0,
                      use_surrogate: bool = False, fp64_band_rel: float = 0.0) -> list:
        """isx_extract of several INRs with the same parameters, run on
        ISX_BATCH_WORKERS streams at once; returns one Mesh per INR."""
        p = _lib.Params(method, precision, float(k), int(max_depth), float(fp64_band), int(max_cells),
                        int(chunk_cells), int(bool(use_surrogate)), 0, float(fp64_band_rel))
        ids = (C.c_int32 * len(mlp_ids))(*[int(i) for i in mlp_ids])
        hs = (C.c_void_p * len(mlp_ids))()
        self._chk(self._L.isx_extract_batch(self._h, len(mlp_ids), ids, C.byref(p), hs))
        return [Mesh(self._L, C.c_void_p(h)) for h in hs]


class Mesh:
    """Library-owned extraction result."""

    def __init__(self, L, h):
        self._L = L
        self._h = h
        nt, nl, nc, nlev = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        L.isx_mesh_info(h, C.byref(nt), C.byref(nl), C.byref(nc), C.byref(nlev))
        self.n_tris, self.n_leaves, self.n_corners, self.n_levels = nt.value, nl.value, nc.value, nlev.value

    def free(self):
        if self._h:
            self._L.isx_mesh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def levels(self):
        out = []
        for i in range(self.n_levels):
            a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
            self._L.isx_mesh_level(self._h, i, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
            x, y = C.c_int64(), C.c_int64()
            self._L.isx_mesh_level_cancelled(self._h, i, C.byref(x))
            self._L.isx_mesh_level_rechecked_fp64(self._h, i, C.byref(y))
            out.append(dict(cells=a.value, active=b.value, rechecked=c.value, propagated=d.value,
                            cancelled=x.value, rechecked_fp64=y.value))
        return out

    def times(self):
        v = [C.c_float() for _ in range(4)]
        self._L.isx_mesh_times(self._h, *[C.byref(x) for x in v])
        return dict(acp_ms=v[0].value, inr_ms=v[1].value, mc_ms=v[2].value, total_ms=v[3].value)

    def triangles(self):
        pos = np.zeros((self.n_tris, 3, 3), dtype=np.float32)
        keys = np.zeros((self.n_tris, 3), dtype=np.uint64)
        iso = np.zeros(self.n_tris, dtype=np.int32)
        st = self._L.isx_mesh_copy_tris(self._h, pos.ctypes.data, keys.ctypes.data, iso.ctypes.data)
        if st != 0:
            raise IsxError(st, "isx_mesh_copy_tris")
        return pos, keys, iso

    def leaves(self):
        ids = np.zeros(self.n_leaves, dtype=np.uint32)
        masks = np.zeros(self.n_leaves, dtype=np.uint32)
        st = self._L.isx_mesh_copy_leaves(self._h, ids.ctypes.data, masks.ctypes.data)
        if st != 0:
            raise IsxError(st, "isx_mesh_copy_leaves")
        return ids, masks

    def level_cells(self, level: int):
        n = self.levels()[level]["cells"]
        ids = np.zeros(n, dtype=np.uint32)
        out = np.zeros((n, 2), dtype=np.float32)
        masks = np.zeros(n, dtype=np.uint32)
        st = self._L.isx_mesh_copy_level(self._h, level, ids.ctypes.data, out.ctypes.data, masks.ctypes.data)
        if st != 0:
            raise IsxError(st, "isx_mesh_copy_level (set KEEP_LEVELS before extracting)")
        return ids, out, masks
