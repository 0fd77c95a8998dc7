"""Thin Python layer over the C ABI: device buffers come from PyTorch, all
work runs in libgavis.so.

    ctx = Context()
    dsc = DeviceScene(scene)                      # attributes resident on the GPU
    gamma = ctx.vf_build(dsc, train_cams, sh_degree=2)
    scores, maps = ctx.vf_query_views(dsc, gamma, 2, train_cams.n, cand_cams)
    best = ctx.select_next_view(scores)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import GV_BF16, GV_F16, GV_F32, check, load

DTYPES = {"f32": GV_F32, "f16": GV_F16, "bf16": GV_BF16}
TORCH_DTYPES = {GV_F32: torch.float32, GV_F16: torch.float16, GV_BF16: torch.bfloat16}


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def half_storage(means: np.ndarray, dtype: str, anchor_block: int = 256):
    """Block-anchored storage of the means: FP32 anchors (block means) and
    half offsets.  Returns (anchors [B,3] f32, offsets [N,3] f16/bf16 tensor,
    dequantised means [N,3] f32 exactly as the kernels rebuild them)."""
    n = means.shape[0]
    nb = (n + anchor_block - 1) // anchor_block
    pad = nb * anchor_block - n
    m = np.concatenate([means, np.repeat(means[-1:], pad, 0)]) if pad else means
    anchors = m.reshape(nb, anchor_block, 3).mean(1).astype(np.float32)
    off = torch.from_numpy(means - np.repeat(anchors, anchor_block, 0)[:n]).to(
        torch.float16 if dtype == "f16" else torch.bfloat16)
    deq = np.repeat(anchors, anchor_block, 0)[:n] + off.float().numpy()
    return anchors, off, deq.astype(np.float32)


class DeviceScene:
    """A scene's Gaussian attributes resident in device memory."""

    def __init__(self, scene, device: str = "cuda", dtype: str = "f32", anchor_block: int = 256):
        self.n = scene.n
        self.n_virtual = int(scene.n_virtual)
        self.dtype = DTYPES[dtype]
        td = TORCH_DTYPES[self.dtype]
        anchors = None
        if self.dtype == GV_F32:
            means = torch.from_numpy(np.ascontiguousarray(scene.means, np.float32))
            self.dequantised_means = scene.means
        else:
            a, means, self.dequantised_means = half_storage(scene.means.astype(np.float32), dtype, anchor_block)
            anchors = torch.from_numpy(a).to(device)
        self.means = means.to(device).contiguous()
        self.scales = torch.from_numpy(np.ascontiguousarray(scene.scales, np.float32)).to(td).to(device).contiguous()
        self.quats = torch.from_numpy(np.ascontiguousarray(scene.quats, np.float32)).to(td).to(device).contiguous()
        self.opacity = torch.from_numpy(np.ascontiguousarray(scene.opacity, np.float32)).to(td).to(device).contiguous()
        self.anchors = anchors
        self.anchor_block = anchor_block
        self.c = _lib.gv_gaussians()
        self.c.n = self.n
        self.c.n_virtual = self.n_virtual
        self.c.dtype = self.dtype
        self.c.means = self.means.data_ptr()
        self.c.scales = self.scales.data_ptr()
        self.c.quats = self.quats.data_ptr()
        self.c.opacity = self.opacity.data_ptr()
        self.c.anchors = anchors.data_ptr() if anchors is not None else None
        self.c.anchor_block = anchor_block if anchors is not None else 0

    def nbytes(self) -> int:
        t = [self.means, self.scales, self.quats, self.opacity] + ([self.anchors] if self.anchors is not None else [])
        return sum(x.numel() * x.element_size() for x in t)


@dataclass
class Workspace:
    plan: _lib.gv_workspace
    buf: torch.Tensor

    @property
    def nbytes(self) -> int:
        return int(self.plan.bytes)


class Context:
    def __init__(self, device: int = 0):
        self.L = load()
        self.device = device
        h = ctypes.c_void_p()
        check(self.L.gv_create(device, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.gv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- plans
    def _alloc(self, plan) -> Workspace:
        buf = torch.empty(max(int(plan.bytes), 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        return Workspace(plan, buf)

    def build_workspace(self, dsc: DeviceScene, cams, params: _lib.gv_vf_params, stream=None) -> Workspace:
        plan = _lib.gv_workspace()
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_build_workspace_size(self.h, ctypes.byref(dsc.c), cc, cams.n, ctypes.byref(params),
                                             ctypes.byref(plan), _stream(stream)))
        return self._alloc(plan)

    def query_plan_exact(self, dsc: DeviceScene, cams, params: _lib.gv_uq_params, sh_degree: int,
                         stream=None) -> _lib.gv_workspace:
        """The exact query workspace plan of `cams` (the library's counting
        pass on the device; synchronises `stream`); allocates nothing."""
        plan = _lib.gv_workspace()
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_query_workspace_size(self.h, ctypes.byref(dsc.c), cc, cams.n, ctypes.byref(params),
                                             sh_degree, ctypes.byref(plan), _stream(stream)))
        return plan

    def query_workspace(self, dsc: DeviceScene, cams, params: _lib.gv_uq_params, sh_degree: int,
                        stream=None, slack: float = 1.0) -> Workspace:
        plan = self.query_plan_exact(dsc, cams, params, sh_degree, stream)
        if slack != 1.0:
            plan.max_records = int(plan.max_records * slack) + 1
            plan.max_instances = int(plan.max_instances * slack) + 1
            plan.bytes = self.L.gv_workspace_bytes(ctypes.byref(plan))
        return self._alloc(plan)

    def query_plan(self, dsc: DeviceScene, cams, sh_degree: int, max_records: int,
                   max_instances: int) -> _lib.gv_workspace:
        """A query workspace plan with caller-chosen capacities, made on the
        host (no device pass): the view, tile and pixel counts of `cams`, and
        the bytes those capacities need.  A call whose records or instances
        exceed them reports GV_ERR_CAPACITY through check_workspace."""
        plan = _lib.gv_workspace()
        wh = np.asarray(cams.wh, dtype=np.int64)
        plan.kind = 1
        plan.n = dsc.n
        plan.sh_degree = int(sh_degree)
        plan.n_views = int(cams.n)
        plan.total_tiles = int(np.sum(((wh[:, 0] + 15) // 16) * ((wh[:, 1] + 15) // 16)))
        plan.total_pixels = int(np.sum(wh[:, 0] * wh[:, 1]))
        plan.max_records = int(max_records)
        plan.max_instances = int(max_instances)
        plan.bytes = self.L.gv_workspace_bytes(ctypes.byref(plan))
        return plan

    def alloc_workspace(self, plan: _lib.gv_workspace) -> Workspace:
        return self._alloc(plan)

    # ---------------------------------------------------------------- calls
    def vf_build(self, dsc: DeviceScene, cams, sh_degree: int = 2, params: Optional[_lib.gv_vf_params] = None,
                 ws: Optional[Workspace] = None, gamma: Optional[torch.Tensor] = None,
                 gamma_dtype: str = "f32", stream=None) -> torch.Tensor:
        if params is None:
            params = _lib.default_vf_params(sh_degree=sh_degree)
        if ws is None:
            ws = self.build_workspace(dsc, cams, params, stream)
        K = (params.sh_degree + 1) ** 2
        gdt = DTYPES[gamma_dtype]
        if gamma is None:
            gamma = torch.empty((K, dsc.n), dtype=TORCH_DTYPES[gdt], device=f"cuda:{self.device}")
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_build(self.h, ctypes.byref(dsc.c), cc, cams.n, ctypes.byref(params), _ptr(gamma), gdt,
                              ctypes.byref(ws.plan), _ptr(ws.buf), _stream(stream)))
        return gamma

    def vf_query_views(self, dsc: DeviceScene, gamma: torch.Tensor, sh_degree: int, n_train: int, cams,
                       params: Optional[_lib.gv_uq_params] = None, ws: Optional[Workspace] = None,
                       want_maps: bool = False, scores: Optional[torch.Tensor] = None,
                       maps: Optional[torch.Tensor] = None, stream=None, want_depth: bool = False):
        """Alg. 4 + Alg. 6 over the candidate views: (scores [n_views], maps).
        maps (with want_maps) packs the entropy maps view after view; with
        want_depth it is twice as long and its second half holds the
        expected-depth maps in the same packing."""
        if params is None:
            params = _lib.default_uq_params()
        want_maps = want_maps or want_depth
        params.write_maps = 1 if want_maps else 0
        params.write_depth = 1 if want_depth else 0
        if ws is None:
            ws = self.query_workspace(dsc, cams, params, sh_degree, stream)
        dev = f"cuda:{self.device}"
        if scores is None:
            scores = torch.empty(cams.n, dtype=torch.float32, device=dev)
        if want_maps and maps is None:
            maps = torch.empty(cams.pixels() * (2 if params.write_depth else 1), dtype=torch.float32, device=dev)
        gdt = {torch.float32: GV_F32, torch.float16: GV_F16, torch.bfloat16: GV_BF16}[gamma.dtype]
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_query_views(self.h, ctypes.byref(dsc.c), _ptr(gamma), gdt, sh_degree, int(n_train), cc,
                                    cams.n, ctypes.byref(params), _ptr(scores), _ptr(maps) if want_maps else None,
                                    ctypes.byref(ws.plan), _ptr(ws.buf), _stream(stream)))
        return scores, maps

    def vf_query_views_noalloc(self, dsc: DeviceScene, gamma: torch.Tensor, sh_degree: int, n_train: int, cams,
                               params: Optional[_lib.gv_uq_params] = None, scores: Optional[torch.Tensor] = None,
                               maps: Optional[torch.Tensor] = None, stream=None):
        """vf_query_views on the library's static per-GPU scratch instead of
        a caller workspace (the call itself allocates no device memory; the
        output tensors are the caller's).  maps, if given, receives the
        entropy maps (and, with params.write_depth, the depth maps)."""
        if params is None:
            params = _lib.default_uq_params()
        params.write_maps = 1 if maps is not None else 0
        if scores is None:
            scores = torch.empty(cams.n, dtype=torch.float32, device=f"cuda:{self.device}")
        gdt = {torch.float32: GV_F32, torch.float16: GV_F16, torch.bfloat16: GV_BF16}[gamma.dtype]
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_query_views_noalloc(self.h, ctypes.byref(dsc.c), _ptr(gamma), gdt, sh_degree, int(n_train),
                                            cc, cams.n, ctypes.byref(params), _ptr(scores), _ptr(maps),
                                            _stream(stream)))
        return scores, maps

    def multiview_visibility(self, dsc: DeviceScene, cams, params: Optional[_lib.gv_vf_params] = None,
                             ws: Optional[Workspace] = None, out: Optional[torch.Tensor] = None,
                             stream=None) -> torch.Tensor:
        """1 - prod_p (1 - v_p[g]) over the views (Alg. 5), float [n]."""
        if params is None:
            params = _lib.default_vf_params()
        if ws is None:
            ws = self.build_workspace(dsc, cams, params, stream)
        if out is None:
            out = torch.empty(dsc.n, dtype=torch.float32, device=f"cuda:{self.device}")
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_multiview_visibility(self.h, ctypes.byref(dsc.c), cc, cams.n, ctypes.byref(params),
                                             _ptr(out), ctypes.byref(ws.plan), _ptr(ws.buf), _stream(stream)))
        return out

    def vf_query_views_color(self, dsc: DeviceScene, gamma: torch.Tensor, sh_degree: int, n_train: int,
                             color_var: torch.Tensor, cams, params: Optional[_lib.gv_uq_params] = None,
                             ws: Optional[Workspace] = None, want_maps: bool = False,
                             scores: Optional[torch.Tensor] = None, maps: Optional[torch.Tensor] = None,
                             stream=None):
        """vf_query_views with the colour covariance of every Gaussian taken
        from the variances of its colour SH coefficients, color_var float32
        [3][Kc][n] (FisherRF integration); same outputs."""
        if params is None:
            params = _lib.default_uq_params()
        params.write_maps = 1 if want_maps else 0
        if color_var.dtype != torch.float32 or color_var.dim() != 3 or color_var.shape[0] != 3 \
                or color_var.shape[2] != dsc.n:
            raise ValueError("color_var must be float32 [3][Kc][n]")
        Lc = int(round(color_var.shape[1] ** 0.5)) - 1
        if (Lc + 1) ** 2 != color_var.shape[1]:
            raise ValueError("color_var's second dimension must be (Lc+1)^2")
        color_var = color_var.contiguous()
        if ws is None:
            ws = self.query_workspace(dsc, cams, params, sh_degree, stream)
        dev = f"cuda:{self.device}"
        if scores is None:
            scores = torch.empty(cams.n, dtype=torch.float32, device=dev)
        if want_maps and maps is None:
            maps = torch.empty(cams.pixels() * (2 if params.write_depth else 1), dtype=torch.float32, device=dev)
        gdt = {torch.float32: GV_F32, torch.float16: GV_F16, torch.bfloat16: GV_BF16}[gamma.dtype]
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_query_views_color(self.h, ctypes.byref(dsc.c), _ptr(gamma), gdt, sh_degree, int(n_train),
                                          _ptr(color_var), Lc, cc, cams.n, ctypes.byref(params), _ptr(scores),
                                          _ptr(maps) if want_maps else None, ctypes.byref(ws.plan), _ptr(ws.buf),
                                          _stream(stream)))
        return scores, maps

    def view_visibility(self, dsc: DeviceScene, cams, params: Optional[_lib.gv_vf_params] = None,
                        ws: Optional[Workspace] = None, stream=None):
        """Per-view single-view visibility v_p[g] (Alg. 2), float [n_views][n],
        and the camera centres, float [n_views][3]: the inputs of
        vf_query_views_exact."""
        if params is None:
            params = _lib.default_vf_params()
        if ws is None:
            ws = self.build_workspace(dsc, cams, params, stream)
        dev = f"cuda:{self.device}"
        vis = torch.empty((cams.n, dsc.n), dtype=torch.float32, device=dev)
        centres = torch.empty((cams.n, 3), dtype=torch.float32, device=dev)
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_view_visibility(self.h, ctypes.byref(dsc.c), cc, cams.n, ctypes.byref(params), _ptr(vis),
                                        _ptr(centres), ctypes.byref(ws.plan), _ptr(ws.buf), _stream(stream)))
        return vis, centres

    def vf_query_views_exact(self, dsc: DeviceScene, view_vis: torch.Tensor, train_centres: torch.Tensor,
                             kappa: float, cams, params: Optional[_lib.gv_uq_params] = None,
                             ws: Optional[Workspace] = None, want_maps: bool = False,
                             scores: Optional[torch.Tensor] = None, maps: Optional[torch.Tensor] = None,
                             stream=None):
        """Alg. 6 with the exact multi-view visibility (eq. vis_all) in place of
        the field's AM-GM query; same outputs as vf_query_views."""
        if params is None:
            params = _lib.default_uq_params()
        params.write_maps = 1 if want_maps else 0
        if view_vis.dtype != torch.float32 or train_centres.dtype != torch.float32:
            raise TypeError("view_vis and train_centres must be float32")
        n_train = int(view_vis.shape[0])
        if tuple(view_vis.shape) != (n_train, dsc.n) or tuple(train_centres.shape) != (n_train, 3):
            raise ValueError("view_vis must be [n_train][n] and train_centres [n_train][3]")
        view_vis, train_centres = view_vis.contiguous(), train_centres.contiguous()
        if ws is None:
            ws = self.query_workspace(dsc, cams, params, 0, stream)
        dev = f"cuda:{self.device}"
        if scores is None:
            scores = torch.empty(cams.n, dtype=torch.float32, device=dev)
        if want_maps and maps is None:
            maps = torch.empty(cams.pixels() * (2 if params.write_depth else 1), dtype=torch.float32, device=dev)
        cc = _lib.cameras_to_c(cams)
        check(self.L.vf_query_views_exact(self.h, ctypes.byref(dsc.c), _ptr(view_vis), _ptr(train_centres),
                                          n_train, float(kappa), cc, cams.n, ctypes.byref(params), _ptr(scores),
                                          _ptr(maps) if want_maps else None, ctypes.byref(ws.plan), _ptr(ws.buf),
                                          _stream(stream)))
        return scores, maps

    def check_workspace(self, ws: Workspace, stream=None):
        """(status, (records, instances, overflow flags, pairs composited))."""
        out = (ctypes.c_int64 * 4)()
        st = self.L.gv_workspace_check(self.h, ctypes.byref(ws.plan), _ptr(ws.buf), out, _stream(stream))
        return st, (int(out[0]), int(out[1]), int(out[2]), int(out[3]))

    def set_tuning(self, vis_batch: int = 64, uq_batch: int = 256, vis_order: int = 2, uq_order: int = 0):
        t = _lib.gv_tuning(vis_batch, uq_batch, vis_order, uq_order)
        check(self.L.gv_set_tuning(self.h, ctypes.byref(t)))

    def get_tuning(self):
        t = _lib.gv_tuning()
        check(self.L.gv_get_tuning(self.h, ctypes.byref(t)))
        return {"vis_batch": t.vis_batch, "uq_batch": t.uq_batch, "vis_order": t.vis_order, "uq_order": t.uq_order}

    def profile(self, on: bool = True):
        check(self.L.gv_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, stream=None) -> dict:
        n = _lib.GV_PROFILE_STAGES
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        check(self.L.gv_profile_read(self.h, ms, calls, _stream(stream)))
        return {self.L.gv_profile_stage_name(i).decode(): (float(ms[i]), int(calls[i])) for i in range(n)}

    def select_next_view(self, scores: torch.Tensor, stream=None) -> int:
        best = ctypes.c_int32(-1)
        check(self.L.select_next_view(self.h, _ptr(scores), int(scores.numel()), ctypes.byref(best),
                                      _stream(stream)))
        return int(best.value)


# ---------------------------------------------------------------- density control (Alg. 5)

def density_control(ctx: "Context", scene, train, u: np.ndarray, lo=None, hi=None, rho: float = 100.0,
                    eta: float = 0.5, eps_v: float = 0.95, params: Optional[_lib.gv_vf_params] = None,
                    device: str = "cuda"):
    """Alg. 5 through the library (vf_density_control): virtual particles in
    the box [lo, hi] (the scene's extent by default) at density rho, from the
    uniform draws u ([n_draw][3] in [0, 1)); the multi-view visibility of the
    scene and the particles; the particles with visibility at most eps_v kept
    as the scene's n_virtual tail.  This function only allocates the device
    arrays (the real attributes copied in, room for the particles behind
    them) and reads the results back.  Returns (augmented scene as a
    scenes.Scene, visibility of every particle, indices of the kept
    particles, N_virt)."""
    from .scenes import Scene
    if params is None:
        params = _lib.default_vf_params()
    ext = scene.extent
    dp = _lib.gv_density_params()
    for k in range(3):
        dp.lo[k] = float(ext[k][0] if lo is None else lo[k])
        dp.hi[k] = float(ext[k][1] if hi is None else hi[k])
    dp.rho, dp.eta, dp.eps_v = float(rho), float(eta), float(eps_v)
    L = load()
    u_dev = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float32)).to(device)
    n_real = int(scene.n)

    def arrays(n_total):
        out = []
        for a, w in ((scene.means, 3), (scene.scales, 3), (scene.quats, 4), (scene.opacity, 1)):
            t = torch.empty((n_total, w) if w > 1 else (n_total,), dtype=torch.float32, device=device)
            t[:n_real] = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
            out.append(t)
        return out

    def gauss(ts, n_total):
        g = _lib.gv_gaussians()
        g.n, g.n_virtual, g.dtype = n_total, 0, GV_F32
        g.means, g.scales, g.quats, g.opacity = (t.data_ptr() for t in ts)
        g.anchors, g.anchor_block = None, 0
        return g

    # N_virt and s come from the library's own arithmetic
    plan = _lib.gv_workspace()
    nv, sc = ctypes.c_int64(0), ctypes.c_float(0.0)
    check(L.vf_virtual_particle_count(ctypes.byref(dp), ctypes.byref(nv), ctypes.byref(sc)))
    n_virt = int(nv.value)
    cc = _lib.cameras_to_c(train)
    ts = arrays(n_real + n_virt)
    g = gauss(ts, n_real + n_virt)
    check(L.vf_density_control_workspace_size(ctx.h, ctypes.byref(g), n_real, _ptr(u_dev), int(u_dev.shape[0]),
                                              ctypes.byref(dp), cc, train.n, ctypes.byref(params),
                                              ctypes.byref(plan), ctypes.byref(nv), _stream(None)))
    ws = ctx.alloc_workspace(plan)
    vis = torch.empty(max(n_real + n_virt, 1), dtype=torch.float32, device=device)
    kept = torch.empty(max(n_virt, 1), dtype=torch.int32, device=device)
    n_kept = ctypes.c_int64(0)
    check(L.vf_density_control(ctx.h, ctypes.byref(g), n_real, _ptr(u_dev), int(u_dev.shape[0]), ctypes.byref(dp),
                               cc, train.n, ctypes.byref(params), _ptr(vis), _ptr(kept), ctypes.byref(n_kept),
                               ctypes.byref(ws.plan), _ptr(ws.buf), _stream(None)))
    k = int(n_kept.value)
    n = n_real + k
    aug = Scene(ts[0][:n].cpu().numpy(), ts[1][:n].cpu().numpy(), ts[2][:n].cpu().numpy(), ts[3][:n].cpu().numpy(),
                k, scene.extent)
    return aug, vis[n_real:n_real + n_virt].cpu().numpy(), kept[:k].cpu().numpy(), n_virt


def split_maps(maps: torch.Tensor, cams):
    """Per-view [h, w] views of the packed maps tensor."""
    out, off = [], 0
    for w, h in cams.wh:
        n = int(w) * int(h)
        out.append(maps[off:off + n].view(int(h), int(w)))
        off += n
    return out
