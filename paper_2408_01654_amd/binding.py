"""ctypes binding of libdpvba.so (include/dpvba.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Tensors must already live on the GPU; torch provides the device
memory and the stream.  There is no CPU fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpvba.so")

DPVBA_OK, DPVBA_EINVAL, DPVBA_ENOTPD, DPVBA_ENOMEM, DPVBA_EHIP, DPVBA_ESTATE, DPVBA_EDEVICE, DPVBA_ELIMIT = range(8)
FP32, MIXED, FP64 = 0, 1, 2
FLAG_GRAPH = 1
FLAG_LEVENBERG = 2          # H + lambda I instead of H + lambda (Diag(H) + I)
FLAG_FORCE_FP64_CHOL = 4    # MIXED: always take the float64 Cholesky
FLAG_NO_REFINE = 8          # MIXED: no refinement steps
MAX_ITERS = 32
PHASES = ("assemble", "gather", "factor", "backsub", "retract", "cost")


class DpvbaError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class Graph(ctypes.Structure):
    _fields_ = [
        ("n_frames", ctypes.c_int32), ("n_patches", ctypes.c_int32), ("n_edges", ctypes.c_int32),
        ("patch_size", ctypes.c_int32), ("n_fixed", ctypes.c_int32),
        ("patches", ctypes.c_void_p), ("ii", ctypes.c_void_p), ("jj", ctypes.c_void_p),
        ("kk", ctypes.c_void_p), ("target", ctypes.c_void_p), ("weight", ctypes.c_void_p),
        ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
    ]


class Opts(ctypes.Structure):
    _fields_ = [("n_iters", ctypes.c_int32), ("precision", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("z_min", ctypes.c_double), ("flags", ctypes.c_uint32)]


class AnalysisInfo(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("n_free", ctypes.c_int32), ("part_S_elems", ctypes.c_int64),
                ("part_vec_elems", ctypes.c_int64), ("grid_cells", ctypes.c_int64), ("u_elems", ctypes.c_int64),
                ("lds_bytes", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_patches_fp32", ctypes.c_int32), ("tile_patches_fp64", ctypes.c_int32),
                ("keep_order", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_iters", ctypes.c_int32),
                ("cost", ctypes.c_double * (MAX_ITERS + 1)),
                ("n_invalid", ctypes.c_int32 * MAX_ITERS),
                ("min_pivot", ctypes.c_double * MAX_ITERS),
                ("refine_resid", ctypes.c_double * MAX_ITERS),
                ("fp64_fallback", ctypes.c_int32 * MAX_ITERS)]

    def to_dict(self):
        n = self.n_iters
        return {"status": int(self.status), "n_iters": n, "cost": list(self.cost[: n + 1]),
                "n_invalid": list(self.n_invalid[:n]), "min_pivot": list(self.min_pivot[:n]),
                "refine_resid": list(self.refine_resid[:n]), "fp64_fallback": list(self.fp64_fallback[:n])}


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2408_01654_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.dpvba_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32]
        L.dpvba_create.restype = ctypes.c_int
        L.dpvba_destroy.argtypes = [vp]
        L.dpvba_destroy.restype = None
        L.dpvba_analyze.argtypes = [vp, ctypes.POINTER(Graph), vp]
        L.dpvba_analyze.restype = ctypes.c_int
        L.dpvba_reproject.argtypes = [vp, ctypes.POINTER(Graph), vp, vp, ctypes.c_float, vp, vp, vp]
        L.dpvba_reproject.restype = ctypes.c_int
        L.dpvba_reduced_system.argtypes = [vp, ctypes.POINTER(Graph), vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp]
        L.dpvba_reduced_system.restype = ctypes.c_int
        L.dpvba_solve.argtypes = [vp, ctypes.POINTER(Graph), vp, vp, ctypes.POINTER(Opts),
                                  ctypes.POINTER(Report), vp]
        L.dpvba_solve.restype = ctypes.c_int
        L.dpvba_solve_noalloc.argtypes = [vp, ctypes.POINTER(Graph), vp, vp, ctypes.POINTER(Opts),
                                          ctypes.POINTER(Report), vp]
        L.dpvba_solve_noalloc.restype = ctypes.c_int
        L.dpvba_proximity_edges.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                            ctypes.c_int32, vp, vp, vp, vp, vp, vp, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), vp]
        L.dpvba_proximity_edges.restype = ctypes.c_int
        L.dpvba_patch_correlation.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32,
                                              vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.dpvba_patch_correlation.restype = ctypes.c_int
        L.dpvba_pgo_sim3.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_uint32, vp, vp, vp]
        L.dpvba_pgo_sim3.restype = ctypes.c_int
        L.dpvba_pgo_apply.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.dpvba_pgo_apply.restype = ctypes.c_int
        L.dpvba_solve_backward.argtypes = [vp, ctypes.POINTER(Graph), vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp,
                                           vp]
        L.dpvba_solve_backward.restype = ctypes.c_int
        L.dpvba_solve_many.argtypes = [ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(Opts), vp, vp]
        L.dpvba_solve_many.restype = ctypes.c_int
        L.dpvba_solve_backward_many.argtypes = [ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(Opts), vp, vp, vp, vp,
                                                vp]
        L.dpvba_solve_backward_many.restype = ctypes.c_int
        L.dpvba_analyze_batch.argtypes = [vp, ctypes.POINTER(Batch), vp, vp]
        L.dpvba_analyze_batch.restype = ctypes.c_int
        L.dpvba_solve_batch.argtypes = [vp, ctypes.POINTER(Batch), vp, vp, ctypes.POINTER(Opts), vp, vp]
        L.dpvba_solve_batch.restype = ctypes.c_int
        L.dpvba_set_cooperative.argtypes = [vp, ctypes.c_int32]
        L.dpvba_set_cooperative.restype = ctypes.c_int
        L.dpvba_trace_begin.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.dpvba_trace_begin.restype = ctypes.c_int
        L.dpvba_trace_end.argtypes = [vp, vp, vp, vp]
        L.dpvba_trace_end.restype = ctypes.c_int
        L.dpvba_analyze_ex.argtypes = [vp, ctypes.POINTER(Graph), ctypes.POINTER(Tuning), vp]
        L.dpvba_analyze_ex.restype = ctypes.c_int
        L.dpvba_get_analysis_info.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(AnalysisInfo)]
        L.dpvba_get_analysis_info.restype = ctypes.c_int
        L.dpvba_get_system_order.argtypes = [vp, vp, ctypes.c_int32]
        L.dpvba_get_system_order.restype = ctypes.c_int
        L.dpvba_last_error.argtypes = [vp]
        L.dpvba_last_error.restype = ctypes.c_char_p
        L.dpvba_status_string.argtypes = [ctypes.c_int]
        L.dpvba_status_string.restype = ctypes.c_char_p
        L.dpvba_device_status.argtypes = [vp, vp, vp]
        L.dpvba_device_status.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().dpvba_status_string(int(s)).decode()


def _check(status: int, what: str, ctx=None):
    if status != DPVBA_OK:
        if ctx is not None and status in (DPVBA_EHIP, DPVBA_ELIMIT):
            what = f"{what} [{lib().dpvba_last_error(ctx).decode()}]"
        raise DpvbaError(status, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class GraphTensors:
    """Device tensors of one BA problem (see dpvba_graph)."""

    n_frames: int
    n_fixed: int
    patches: torch.Tensor   # [P,p,p,2] float32
    ii: torch.Tensor        # [E] int32
    jj: torch.Tensor
    kk: torch.Tensor
    target: torch.Tensor    # [E,2] float32
    weight: torch.Tensor    # [E,2] float32
    intrinsics: tuple       # fx, fy, cx, cy

    @staticmethod
    def from_arrays(n_frames, n_fixed, patches, ii, jj, kk, target, weight, intrinsics, device="cuda"):
        f32 = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        i32 = lambda a: torch.as_tensor(a).to(device=device, dtype=torch.int32).contiguous()
        return GraphTensors(int(n_frames), int(n_fixed), f32(patches), i32(ii), i32(jj), i32(kk),
                            f32(target).reshape(-1, 2), f32(weight).reshape(-1, 2),
                            tuple(float(x) for x in intrinsics))

    @staticmethod
    def from_scene(scene, device="cuda"):
        return GraphTensors.from_arrays(scene.n_frames, scene.n_fixed, scene.patches, scene.ii, scene.jj,
                                        scene.kk, scene.target, scene.weight, scene.intrinsics, device)

    def struct(self) -> Graph:
        fx, fy, cx, cy = self.intrinsics
        return Graph(self.n_frames, self.patches.shape[0], self.ii.shape[0], self.patches.shape[1],
                     self.n_fixed, _ptr(self.patches), _ptr(self.ii), _ptr(self.jj), _ptr(self.kk),
                     _ptr(self.target), _ptr(self.weight), fx, fy, cx, cy)


class Batch(ctypes.Structure):
    _fields_ = [
        ("n_problems", ctypes.c_int32), ("patch_size", ctypes.c_int32),
        ("frame_off", ctypes.c_void_p), ("patch_off", ctypes.c_void_p), ("edge_off", ctypes.c_void_p),
        ("n_fixed", ctypes.c_void_p), ("patches", ctypes.c_void_p), ("ii", ctypes.c_void_p),
        ("jj", ctypes.c_void_p), ("kk", ctypes.c_void_p), ("target", ctypes.c_void_p), ("weight", ctypes.c_void_p),
        ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
    ]


@dataclass
class BatchTensors:
    """Device tensors of a batch of problems packed back to back (see
    dpvba_batch); indices are local to each problem."""

    frame_off: np.ndarray   # host int32 [B+1]
    patch_off: np.ndarray
    edge_off: np.ndarray
    n_fixed: np.ndarray     # host int32 [B]
    patches: torch.Tensor   # [sum P,p,p,2] float32
    ii: torch.Tensor        # [sum E] int32
    jj: torch.Tensor
    kk: torch.Tensor
    target: torch.Tensor    # [sum E,2] float32
    weight: torch.Tensor
    intrinsics: tuple
    poses: torch.Tensor     # [sum N,7] float32 starting poses
    inv_depth: torch.Tensor  # [sum P] float32 starting inverse depths

    @property
    def n_problems(self) -> int:
        return len(self.n_fixed)

    @staticmethod
    def from_scenes(scenes, device="cuda"):
        """Pack scenes (one camera) into one batch."""
        intr = tuple(float(x) for x in scenes[0].intrinsics)
        for s in scenes:
            if tuple(float(x) for x in s.intrinsics) != intr:
                raise ValueError("a batch has one camera")
        cat = lambda name: np.concatenate([getattr(s, name) for s in scenes], 0)
        off = lambda xs: np.concatenate([[0], np.cumsum(xs)]).astype(np.int32)
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(device)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32).to(device)
        return BatchTensors(
            off([s.n_frames for s in scenes]), off([s.n_patches for s in scenes]), off([s.n_edges for s in scenes]),
            np.array([s.n_fixed for s in scenes], dtype=np.int32), f32(cat("patches")), i32(cat("ii")),
            i32(cat("jj")), i32(cat("kk")), f32(cat("target")).reshape(-1, 2), f32(cat("weight")).reshape(-1, 2),
            intr, f32(cat("poses")), f32(cat("inv_depth")))

    def struct(self) -> Batch:
        fx, fy, cx, cy = self.intrinsics
        self._host = [np.ascontiguousarray(a, dtype=np.int32) for a in
                      (self.frame_off, self.patch_off, self.edge_off, self.n_fixed)]
        hp = [a.ctypes.data_as(ctypes.c_void_p) for a in self._host]
        return Batch(self.n_problems, self.patches.shape[1], hp[0], hp[1], hp[2], hp[3], _ptr(self.patches),
                     _ptr(self.ii), _ptr(self.jj), _ptr(self.kk), _ptr(self.target), _ptr(self.weight),
                     fx, fy, cx, cy)


class Context:
    """One dpvba_ctx on a device."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p(0)
        _check(lib().dpvba_create(ctypes.byref(self._h), int(device)), "dpvba_create")
        self.device = device
        self._graph = None

    def close(self):
        if self._h:
            lib().dpvba_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def analyze(self, g: GraphTensors, stream=None, tile_patches_fp32=0, tile_patches_fp64=0, keep_order=False):
        gs = g.struct()
        tune = Tuning(int(tile_patches_fp32), int(tile_patches_fp64), int(bool(keep_order)))
        _check(lib().dpvba_analyze_ex(self._h, ctypes.byref(gs), ctypes.byref(tune), _stream(stream)),
               "dpvba_analyze", self._h)
        self._graph = g

    def analysis_info(self, precision=FP32) -> dict:
        info = AnalysisInfo()
        _check(lib().dpvba_get_analysis_info(self._h, int(precision), ctypes.byref(info)), "dpvba_get_analysis_info")
        return {f: getattr(info, f) for f, _ in AnalysisInfo._fields_}

    def system_order(self) -> np.ndarray:
        """dpvba_get_system_order: free pose at each block row of the factor."""
        n = int(self.analysis_info()["n_free"])
        out = np.zeros(max(n, 1), dtype=np.int32)
        _check(lib().dpvba_get_system_order(self._h, out.ctypes.data_as(ctypes.c_void_p), n),
               "dpvba_get_system_order", self._h)
        return out[:n]

    def pgo_sim3(self, poses, loop_j, loop_k, loop_rel, n_fixed=1, n_iters=10, lam=1e-4, levenberg=False,
                 stream=None):
        """Sim(3) pose-graph optimisation (dpvba_pgo_sim3): poses [N,7] and
        loop_rel [L,8] float64 on the device, loop_j / loop_k host int
        sequences.  Returns (sims [N,8] float64 device, costs list)."""
        n = int(poses.shape[0])
        lj = np.ascontiguousarray(np.asarray(loop_j, dtype=np.int32))
        lk = np.ascontiguousarray(np.asarray(loop_k, dtype=np.int32))
        sims = torch.empty((n, 8), dtype=torch.float64, device=poses.device)
        cost = (ctypes.c_double * (int(n_iters) + 1))()
        st = lib().dpvba_pgo_sim3(self._h, n, int(n_fixed), _ptr(poses), len(lj),
                                  lj.ctypes.data_as(ctypes.c_void_p), lk.ctypes.data_as(ctypes.c_void_p),
                                  _ptr(loop_rel) if len(lj) else None, int(n_iters), float(lam),
                                  FLAG_LEVENBERG if levenberg else 0, _ptr(sims), ctypes.cast(cost, ctypes.c_void_p),
                                  _stream(stream))
        _check(st, "dpvba_pgo_sim3", self._h)
        return sims, list(cost)

    def pgo_apply(self, sims, patch_off, poses, inv_depth, stream=None):
        """G_i <- (t_i, R_i), d <- d / s_i in place (dpvba_pgo_apply)."""
        _check(lib().dpvba_pgo_apply(self._h, int(sims.shape[0]), _ptr(sims), _ptr(patch_off), _ptr(poses),
                                     _ptr(inv_depth), _stream(stream)), "dpvba_pgo_apply", self._h)

    def patch_correlation(self, gmap, fmaps, kk, jj, coords, out=None, stream=None):
        """corr [E, p, p, 7, 7] of eq. 4 (dpvba_patch_correlation): gmap
        [P, p, p, D], fmaps [M, H, W, D] float32, kk / jj [E] int32, coords
        [E, p, p, 2] float32, all on the device."""
        E, p = int(coords.shape[0]), int(coords.shape[1])
        D = int(gmap.shape[-1])
        corr = out if out is not None else torch.empty((E, p, p, 7, 7), dtype=torch.float32, device=coords.device)
        _check(lib().dpvba_patch_correlation(self._h, E, p, D, _ptr(gmap), int(gmap.shape[0]), _ptr(fmaps),
                                             int(fmaps.shape[0]), int(fmaps.shape[1]), int(fmaps.shape[2]), _ptr(kk),
                                             _ptr(jj), _ptr(coords), _ptr(corr), _stream(stream)),
               "dpvba_patch_correlation", self._h)
        return corr

    def proximity_edges(self, poses, patch_off, first_recent=0, min_gap=100, radius=2.0, max_targets=10,
                        stream=None):
        """Loop-closure edges by camera proximity (dpvba_proximity_edges).
        poses [N,7] float32 and patch_off [N+1] int32 on the device.  Returns
        (counts [N], targets [N,max_targets], edge_off [N+1], ii, jj, kk)."""
        n = int(poses.shape[0])
        dev = poses.device
        counts = torch.empty((n,), dtype=torch.int32, device=dev)
        targets = torch.empty((n, max(1, max_targets)), dtype=torch.int32, device=dev)
        edge_off = torch.empty((n + 1,), dtype=torch.int64, device=dev)
        cap = int(patch_off[-1].item()) * int(max_targets)
        ii = torch.empty((max(1, cap),), dtype=torch.int32, device=dev)
        jj = torch.empty_like(ii)
        kk = torch.empty_like(ii)
        ne = ctypes.c_int64(0)
        _check(lib().dpvba_proximity_edges(self._h, _ptr(poses), n, _ptr(patch_off), int(first_recent), int(min_gap),
                                           float(radius), int(max_targets), _ptr(counts), _ptr(targets),
                                           _ptr(edge_off), _ptr(ii), _ptr(jj), _ptr(kk), cap, ctypes.byref(ne),
                                           _stream(stream)), "dpvba_proximity_edges", self._h)
        m = int(ne.value)
        return counts, targets[:, :max_targets], edge_off, ii[:m], jj[:m], kk[:m]

    def reproject(self, g: GraphTensors, poses, inv_depth, z_min=0.1, stream=None):
        E, p = g.ii.shape[0], g.patches.shape[1]
        coords = torch.empty((E, p, p, 2), dtype=torch.float32, device=poses.device)
        valid = torch.empty((E,), dtype=torch.uint8, device=poses.device)
        gs = g.struct()
        _check(lib().dpvba_reproject(self._h, ctypes.byref(gs), _ptr(poses), _ptr(inv_depth), float(z_min),
                                     _ptr(coords), _ptr(valid), _stream(stream)), "dpvba_reproject", self._h)
        return coords, valid

    @staticmethod
    def _opts(n_iters, lam, z_min, precision, flags=0):
        return Opts(int(n_iters), int(precision), float(lam), float(z_min), int(flags))

    def device_status(self, stream=None):
        """Synchronise the stream and return (status, cause bits) of the
        device-side failures recorded since the last call; clears them."""
        cause = ctypes.c_int32(0)
        st = lib().dpvba_device_status(self._h, _stream(stream), ctypes.byref(cause))
        if st not in (DPVBA_OK, DPVBA_EDEVICE):
            _check(st, "dpvba_device_status", self._h)
        return st, int(cause.value)

    def reduced_system(self, g: GraphTensors, poses, inv_depth, lam=1e-4, z_min=0.1, precision=FP32,
                       stream=None, flags=0):
        """S [n,n] and s [n] at (poses, inv_depth); float64 for FP64 and
        MIXED (float32 assembly gathered in float64), else float32."""
        dt = torch.float64 if precision in (FP64, MIXED) else torch.float32
        n = 6 * (g.n_frames - g.n_fixed)
        S = torch.empty((n, n), dtype=dt, device=poses.device)
        s = torch.empty((n,), dtype=dt, device=poses.device)
        cost = torch.empty((1,), dtype=torch.float64, device=poses.device)
        o = self._opts(0, lam, z_min, precision, flags)
        gs = g.struct()
        _check(lib().dpvba_reduced_system(self._h, ctypes.byref(gs), _ptr(poses), _ptr(inv_depth),
                                          ctypes.byref(o), _ptr(S), _ptr(s), _ptr(cost), _stream(stream)),
               "dpvba_reduced_system", self._h)
        return S, s, cost

    def solve(self, g: GraphTensors, poses, inv_depth, n_iters=2, lam=1e-4, z_min=0.1, precision=FP32,
              report=True, stream=None, flags=0, noalloc=False):
        """In-place solve of poses [N,7] and inv_depth [P] (float32 for FP32 and
        MIXED, float64 for FP64).  Returns the report as a dict (after
        synchronising the stream) or None.  noalloc=True calls
        dpvba_solve_noalloc (per-call buffers in the library's static device
        array) instead of dpvba_solve."""
        want = torch.float64 if precision == FP64 else torch.float32
        if poses.dtype != want or inv_depth.dtype != want:
            raise TypeError(f"poses and inv_depth must be {want}")
        if not (poses.is_contiguous() and inv_depth.is_contiguous()):
            raise ValueError("poses and inv_depth must be contiguous")
        o = self._opts(n_iters, lam, z_min, precision, flags)
        gs = g.struct()
        rep = Report() if report else None
        fn, name = (lib().dpvba_solve_noalloc, "dpvba_solve_noalloc") if noalloc else (lib().dpvba_solve, "dpvba_solve")
        _check(fn(self._h, ctypes.byref(gs), _ptr(poses), _ptr(inv_depth), ctypes.byref(o),
                  ctypes.byref(rep) if rep is not None else None, _stream(stream)), name, self._h)
        if rep is None:
            return None
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        return rep.to_dict()

    def solve_backward(self, g: GraphTensors, poses0, inv_depth0, grad_poses=None, grad_inv_depth=None, n_iters=2,
                       lam=1e-4, z_min=0.1, precision=FP32, stream=None, flags=0):
        """Gradients (target [E,2], weight [E,2]) of a loss whose gradients
        with respect to the poses and inverse depths that `solve` returns
        from (poses0, inv_depth0) are grad_poses [N,7] and grad_inv_depth [P]
        (either may be None for zero).  All float32, or float64 for FP64."""
        want = torch.float64 if precision == FP64 else torch.float32
        for name, t in (("poses0", poses0), ("inv_depth0", inv_depth0), ("grad_poses", grad_poses),
                        ("grad_inv_depth", grad_inv_depth)):
            if t is not None and (t.dtype != want or not t.is_contiguous()):
                raise TypeError(f"{name} must be a contiguous {want} tensor")
        E = g.ii.shape[0]
        gt = torch.empty((E, 2), dtype=want, device=poses0.device)
        gw = torch.empty((E, 2), dtype=want, device=poses0.device)
        o = self._opts(n_iters, lam, z_min, precision, flags)
        gs = g.struct()
        _check(lib().dpvba_solve_backward(self._h, ctypes.byref(gs), _ptr(poses0), _ptr(inv_depth0), ctypes.byref(o),
                                          _ptr(grad_poses), _ptr(grad_inv_depth), _ptr(gt), _ptr(gw),
                                          _stream(stream)), "dpvba_solve_backward", self._h)
        return gt, gw

    def analyze_batch(self, b: "BatchTensors", tile_patches=None, stream=None):
        """Symbolic analysis of a packed batch; tile_patches: per-problem
        patches per tile (float32 / mixed) or None for the default."""
        bs = b.struct()
        tp = None
        if tile_patches is not None:
            self._tp = np.ascontiguousarray(tile_patches, dtype=np.int32)
            if self._tp.shape != (b.n_problems,):
                raise ValueError("tile_patches must have one entry per problem")
            tp = self._tp.ctypes.data_as(ctypes.c_void_p)
        _check(lib().dpvba_analyze_batch(self._h, ctypes.byref(bs), tp, _stream(stream)), "dpvba_analyze_batch",
               self._h)

    def solve_batch(self, b: "BatchTensors", poses, inv_depth, n_iters=2, lam=1e-4, z_min=0.1, precision=FP32,
                    report=True, graph=False, stream=None, flags=0):
        """In-place solve of every problem of an analysed batch: poses
        [sum N,7], inv_depth [sum P] (float32 for FP32 / MIXED, float64 for
        FP64).  graph=True records the launches in a HIP graph on first use
        and replays it.  Returns the per-problem reports (after synchronising
        the stream) or None."""
        want = torch.float64 if precision == FP64 else torch.float32
        if poses.dtype != want or inv_depth.dtype != want:
            raise TypeError(f"poses and inv_depth must be {want}")
        if not (poses.is_contiguous() and inv_depth.is_contiguous()):
            raise ValueError("poses and inv_depth must be contiguous")
        bs = b.struct()
        o = Opts(int(n_iters), int(precision), float(lam), float(z_min), (FLAG_GRAPH if graph else 0) | int(flags))
        reps = (Report * b.n_problems)() if report else None
        _check(lib().dpvba_solve_batch(self._h, ctypes.byref(bs), _ptr(poses), _ptr(inv_depth), ctypes.byref(o),
                                       ctypes.cast(reps, ctypes.c_void_p) if reps is not None else None,
                                       _stream(stream)), "dpvba_solve_batch", self._h)
        if reps is None:
            return None
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        return [r.to_dict() for r in reps]

    def set_cooperative(self, cooperative: bool):
        """Cooperative (True) or ordinary (False, the default) launch of the
        single-launch small-system solver; results are identical."""
        _check(lib().dpvba_set_cooperative(self._h, int(bool(cooperative))), "dpvba_set_cooperative", self._h)

    def trace_begin(self, sample_every: int = 1, max_pairs: int = 1 << 16):
        _check(lib().dpvba_trace_begin(self._h, int(sample_every), int(max_pairs)), "dpvba_trace_begin", self._h)

    def trace_end(self):
        """Per phase: (summed ms of sampled launches, sampled count, launches seen)."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        ns = (ctypes.c_int32 * n)()
        nl = (ctypes.c_int64 * n)()
        _check(lib().dpvba_trace_end(self._h, ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(ns, ctypes.c_void_p),
                                     ctypes.cast(nl, ctypes.c_void_p)), "dpvba_trace_end", self._h)
        return {PHASES[p]: (ms[p], ns[p], nl[p]) for p in range(n)}


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[_ptr(t).value if t is not None else None for t in ts])


def _many_args(contexts, graphs):
    if len(contexts) != len(graphs) or not contexts:
        raise ValueError("one graph per context, at least one")
    hs = (ctypes.c_void_p * len(contexts))(*[c._h for c in contexts])
    gs = (Graph * len(graphs))(*[g.struct() for g in graphs])
    return hs, gs


def solve_many(contexts, graphs, poses, inv_depth, n_iters=2, lam=1e-4, z_min=0.1, precision=FP32, stream=None,
               flags=0):
    """dpvba_solve_many: in-place solves of several analysed problems
    (contexts[i] analysed for graphs[i]; poses[i], inv_depth[i] as for
    Context.solve), run concurrently; no reports."""
    want = torch.float64 if precision == FP64 else torch.float32
    for t in list(poses) + list(inv_depth):
        if t.dtype != want or not t.is_contiguous():
            raise TypeError(f"poses and inv_depth must be contiguous {want} tensors")
    hs, gs = _many_args(contexts, graphs)
    o = Context._opts(n_iters, lam, z_min, precision, flags)
    _check(lib().dpvba_solve_many(len(contexts), hs, gs, _ptrs(poses), _ptrs(inv_depth), ctypes.byref(o), None,
                                  _stream(stream)), "dpvba_solve_many", contexts[0]._h)


def solve_backward_many(contexts, graphs, poses0, inv_depth0, grad_poses=None, grad_inv_depth=None, n_iters=2,
                        lam=1e-4, z_min=0.1, precision=FP32, stream=None, flags=0):
    """dpvba_solve_backward_many: Context.solve_backward of several problems,
    run concurrently.  grad_poses / grad_inv_depth: lists (entries may be
    None) or None.  Returns the lists of (grad_target, grad_weight)."""
    want = torch.float64 if precision == FP64 else torch.float32
    n = len(contexts)
    gp = [None] * n if grad_poses is None else list(grad_poses)
    gd = [None] * n if grad_inv_depth is None else list(grad_inv_depth)
    for t in list(poses0) + list(inv_depth0) + gp + gd:
        if t is not None and (t.dtype != want or not t.is_contiguous()):
            raise TypeError(f"all arrays must be contiguous {want} tensors")
    hs, gs = _many_args(contexts, graphs)
    gt = [torch.empty((g.ii.shape[0], 2), dtype=want, device=p.device) for g, p in zip(graphs, poses0)]
    gw = [torch.empty_like(t) for t in gt]
    o = Context._opts(n_iters, lam, z_min, precision, flags)
    _check(lib().dpvba_solve_backward_many(n, hs, gs, _ptrs(poses0), _ptrs(inv_depth0), ctypes.byref(o), _ptrs(gp),
                                           _ptrs(gd), _ptrs(gt), _ptrs(gw), _stream(stream)),
           "dpvba_solve_backward_many", contexts[0]._h)
    return gt, gw


class _BundleAdjust(torch.autograd.Function):
    """(target, weight) -> (poses, inv_depth) after n_iters iterations, with
    the adjoint of the unrolled iterations as its backward."""

    @staticmethod
    def forward(ctx, target, weight, poses0, inv_depth0, context, graph, n_iters, lam, z_min, precision):
        dt = torch.float64 if precision == FP64 else torch.float32
        g = GraphTensors(graph.n_frames, graph.n_fixed, graph.patches, graph.ii, graph.jj, graph.kk,
                         target.detach().to(torch.float32).contiguous(),
                         weight.detach().to(torch.float32).contiguous(), graph.intrinsics)
        p0 = poses0.detach().to(dt).contiguous()
        d0 = inv_depth0.detach().to(dt).contiguous()
        poses, d = p0.clone(), d0.clone()
        context.solve(g, poses, d, n_iters, lam, z_min, precision, report=False)
        ctx.save_for_backward(p0, d0)
        ctx.g, ctx.context = g, context
        ctx.args = (n_iters, lam, z_min, precision)
        ctx.dtypes = (target.dtype, weight.dtype)
        return poses, d

    @staticmethod
    def backward(ctx, grad_poses, grad_d):
        p0, d0 = ctx.saved_tensors
        n_iters, lam, z_min, precision = ctx.args
        gp = None if grad_poses is None else grad_poses.to(p0.dtype).contiguous()
        gd = None if grad_d is None else grad_d.to(d0.dtype).contiguous()
        gt, gw = ctx.context.solve_backward(ctx.g, p0, d0, gp, gd, n_iters, lam, z_min, precision)
        return gt.to(ctx.dtypes[0]), gw.to(ctx.dtypes[1]), None, None, None, None, None, None, None, None


def bundle_adjust(context: Context, graph: GraphTensors, poses0, inv_depth0, target, weight, n_iters=2, lam=1e-4,
                  z_min=0.1, precision=FP32):
    """Differentiable BA layer: the poses [N,7] and inverse depths [P] after
    n_iters Gauss-Newton iterations from (poses0, inv_depth0), differentiable
    with respect to target [E,2] and weight [E,2].  `context` must have
    analysed `graph` (its index arrays); the graph's own target and weight
    are not used.  Forward and backward run in libdpvba.so."""
    return _BundleAdjust.apply(target, weight, poses0, inv_depth0, context, graph, n_iters, lam, z_min, precision)


class _BundleAdjustMany(torch.autograd.Function):
    """bundle_adjust over several problems: the forwards run one after
    another on the current stream (ordinary launches: a small problem's
    single-launch solver is fastest alone), the adjoints concurrently
    (dpvba_solve_backward_many).  Inputs: the per-problem targets and
    weights, then the starting points; outputs: poses and inverse depths of
    every problem."""

    @staticmethod
    def forward(ctx, meta, *tensors):
        contexts, graphs, n_iters, lam, z_min, precision = meta
        n = len(contexts)
        dt = torch.float64 if precision == FP64 else torch.float32
        tg, wg, p0, d0 = tensors[:n], tensors[n:2 * n], tensors[2 * n:3 * n], tensors[3 * n:]
        gs = [GraphTensors(g.n_frames, g.n_fixed, g.patches, g.ii, g.jj, g.kk,
                           t.detach().to(torch.float32).contiguous(), w.detach().to(torch.float32).contiguous(),
                           g.intrinsics) for g, t, w in zip(graphs, tg, wg)]
        p0 = [p.detach().to(dt).contiguous() for p in p0]
        d0 = [d.detach().to(dt).contiguous() for d in d0]
        poses, ds = [p.clone() for p in p0], [d.clone() for d in d0]
        for c, g, p, d in zip(contexts, gs, poses, ds):
            c.solve(g, p, d, n_iters, lam, z_min, precision, report=False)
        ctx.save_for_backward(*p0, *d0)
        ctx.gs, ctx.contexts, ctx.args = gs, contexts, (n_iters, lam, z_min, precision)
        ctx.dtypes = [(t.dtype, w.dtype) for t, w in zip(tg, wg)]
        return (*poses, *ds)

    @staticmethod
    def backward(ctx, *grads):
        n = len(ctx.contexts)
        saved = ctx.saved_tensors
        p0, d0 = list(saved[:n]), list(saved[n:])
        gp = [None if g is None else g.to(p.dtype).contiguous() for g, p in zip(grads[:n], p0)]
        gd = [None if g is None else g.to(d.dtype).contiguous() for g, d in zip(grads[n:], d0)]
        gt, gw = solve_backward_many(ctx.contexts, ctx.gs, p0, d0, gp, gd, *ctx.args)
        gt = [t.to(dt[0]) for t, dt in zip(gt, ctx.dtypes)]
        gw = [w.to(dt[1]) for w, dt in zip(gw, ctx.dtypes)]
        return (None, *gt, *gw, *([None] * (2 * n)))


def bundle_adjust_many(contexts, graphs, poses0, inv_depth0, targets, weights, n_iters=2, lam=1e-4, z_min=0.1,
                       precision=FP32):
    """bundle_adjust for several problems at once (contexts[i] has analysed
    graphs[i]): returns the lists of poses and inverse depths; the backward
    runs the problems' adjoints concurrently."""
    n = len(contexts)
    out = _BundleAdjustMany.apply((list(contexts), list(graphs), n_iters, lam, z_min, precision), *targets, *weights,
                                  *poses0, *inv_depth0)
    return list(out[:n]), list(out[n:])
