"""ctypes binding of libkbmi.so: argument marshalling only.

Every step of the search runs inside the HIP library.  This module turns
torch device tensors into pointers, passes torch's current HIP stream, and
raises KbError with the library's message for any non-OK status.  There is no
fallback: if libkbmi.so is missing, loading fails with an ImportError.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkbmi.so")

KB_OK, KB_EINVAL, KB_ENOMEM, KB_EDEVICE, KB_EUNSUPPORTED = 0, -1, -2, -3, -4
KB_F32, KB_F16, KB_BF16 = 0, 1, 2
_STATUS = {0: "KB_OK", -1: "KB_EINVAL", -2: "KB_ENOMEM", -3: "KB_EDEVICE", -4: "KB_EUNSUPPORTED"}

_lock = threading.Lock()
_lib = None

_p, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_SIGNATURES = {
    "kb_abi_version": (ctypes.c_int, []),
    "kb_last_error": (ctypes.c_char_p, []),
    "kb_displacements": (ctypes.c_int, [_p, _i64, _p, _i64, _p]),
    "kb_make_psi_phi": (ctypes.c_int, [_p, _p, _p, _i64, _i64, _i64, _p, _i64, _i64, _p, _i32,
                                       _p, _p, _p]),
    "kb_search_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64]),
    "kb_mask_bright": (ctypes.c_int, [_p, _p, _i64, _i64, _i64, ctypes.c_float, _p]),
    "kb_search": (ctypes.c_int, [_p, _i32, _p, _i64, _i64, _i64, _p, _p, _i64, _i64, _p, _p, _p,
                                 _p, _p, _sz, _p]),
    "kb_topk": (ctypes.c_int, [_p, _i64, _i64, _i64, _p, _p, _i64, _p, _p, _p, _p, _i64, _i64,
                               _p, _p, _p, _p, _p, _sz, _p]),
    "kb_lightcurve_filter": (ctypes.c_int, [_p, _i64, _i64, _i64, _p, _p, _i64, _p, _i64,
                                            ctypes.c_double, ctypes.c_double, _p, _p, _p, _p, _p,
                                            _sz, _p]),
    "kb_search_threshold": (ctypes.c_int, [_p, _i64, _i64, _i64, _p, _p, _i64, ctypes.c_float,
                                           _p, _i64, _p, _p, _sz, _p]),
    "kb_cluster_workspace_bytes": (_sz, [_i64, _i64]),
    "kb_cluster_hits": (ctypes.c_int, [_p, _i64, _p, _i64, ctypes.c_double, ctypes.c_double, _p,
                                       _p, _sz, _p]),
    "kb_stamps": (ctypes.c_int, [_p, _p, _p, _i64, _i64, _i64, _p, _p, _i64, _p, _p, _i64,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _p, _p, _p, _p, _sz, _p]),
    "kb_search_batch_workspace_bytes": (_sz, [_p, _i64]),
    "kb_search_batch": (ctypes.c_int, [_p, _i64, _i32, _i64, _p, _sz, _p]),
    "kb_search_noalloc": (ctypes.c_int, [_p, _i32, _p, _i64, _i64, _i64, _p, _p, _i64, _i64, _p,
                                         _p, _p, _p, _p]),
}


class KbJob(ctypes.Structure):
    """Mirror of the C struct kb_job (one stack of a batched search)."""
    _fields_ = [("planes", _p), ("lp_scale", _p), ("n_img", _i64), ("h", _i64), ("w", _i64),
                ("t", _p), ("vel", _p), ("n_vel", _i64), ("cand_nu", _p), ("cand_alpha", _p),
                ("cand_vel", _p), ("cand_nobs", _p)]


class KbError(RuntimeError):
    """A libkbmi call returned a non-OK status."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libkbmi.so once; raises ImportError if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_1901_02492_amd.build`")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(status: int) -> None:
    if status != KB_OK:
        raise KbError(status, load().kb_last_error().decode())


def _host_f64(a, shape_last=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def displacements(t, vel) -> np.ndarray:
    """Host table int32 [V][N][2] of the offsets every kernel uses."""
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    out = np.empty((vel.shape[0], t.size, 2), dtype=np.int32)
    _check(load().kb_displacements(t.ctypes.data, t.size, vel.ctypes.data, vel.shape[0],
                                   out.ctypes.data))
    return out


def search_workspace_bytes(n_img: int, h: int, w: int, n_vel: int) -> int:
    return int(load().kb_search_workspace_bytes(n_img, h, w, n_vel))


# ---------------------------------------------------------------------------
# Device calls (torch tensors on a HIP device).
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


_LP = {"f16": KB_F16, "bf16": KB_BF16}


def _lp_torch_dtype(code):
    torch = _torch()
    return torch.float16 if code == KB_F16 else torch.bfloat16


def mask_bright(img, mask, threshold, stream=None):
    """kb_mask_bright: mask |= img > threshold, in place; returns mask."""
    torch = _torch()
    n, h, w = img.shape
    if tuple(mask.shape) != (n, h, w):
        raise ValueError("mask must have the image stack's shape")
    _check(load().kb_mask_bright(_dev(img, torch.float32, "img"), _dev(mask, torch.uint8, "mask"),
                                 n, h, w, float(threshold), _stream(stream)))
    return mask


def make_psi_phi(img, var, mask, psf, out=None, stream=None, lp=None, lp_out=None,
                 lp_scale=None):
    """psi/phi planes float32 [N][H][W][2] from device img, var (float32) and
    mask (uint8 or None); psf is a host float32 [ph][pw] array.

    With lp="f16" or "bf16" also writes the scaled 16-bit copy and returns
    (planes, lp_planes [N][H][W][2] float16/bfloat16, scale float32 [N][2])."""
    torch = _torch()
    n, h, w = img.shape
    psf = np.ascontiguousarray(np.asarray(psf, dtype=np.float32))
    if out is None:
        out = torch.empty((n, h, w, 2), dtype=torch.float32, device=img.device)
    code = KB_F32 if lp is None else _LP[lp]
    lp_ptr = sc_ptr = None
    if code != KB_F32:
        if lp_out is None:
            lp_out = torch.empty((n, h, w, 2), dtype=_lp_torch_dtype(code), device=img.device)
        if lp_scale is None:
            lp_scale = torch.empty((n, 2), dtype=torch.float32, device=img.device)
        lp_ptr = _dev(lp_out, _lp_torch_dtype(code), "psi_phi_lp")
        sc_ptr = _dev(lp_scale, torch.float32, "lp_scale")
    mp = 0 if mask is None else _dev(mask, torch.uint8, "mask")
    _check(load().kb_make_psi_phi(_dev(img, torch.float32, "img"),
                                  _dev(var, torch.float32, "var"), mp or None, n, h, w,
                                  psf.ctypes.data, psf.shape[0], psf.shape[1],
                                  _dev(out, torch.float32, "psi_phi"), code, lp_ptr, sc_ptr,
                                  _stream(stream)))
    return out if code == KB_F32 else (out, lp_out, lp_scale)


def alloc_candidates(h, w, k, device):
    torch = _torch()
    return (torch.empty((h, w, k), dtype=torch.float32, device=device),
            torch.empty((h, w, k), dtype=torch.float32, device=device),
            torch.empty((h, w, k), dtype=torch.int32, device=device),
            torch.empty((h, w, k), dtype=torch.int16, device=device))


def alloc_workspace(n_img, h, w, n_vel, device):
    torch = _torch()
    nb = search_workspace_bytes(n_img, h, w, n_vel)
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)


def search(planes, t, vel, k_cand, out=None, workspace=None, stream=None, lp_scale=None):
    """kb_search on planes [N][H][W][2] (float32, or float16 / bfloat16 with
    their lp_scale); returns (nu, alpha, vel, nobs) candidate tensors
    [H][W][k_cand], each pixel's candidates in rank order."""
    torch = _torch()
    n, h, w, two = planes.shape
    assert two == 2
    code = {torch.float32: KB_F32, torch.float16: KB_F16, torch.bfloat16: KB_BF16}[planes.dtype]
    sc_ptr = None if code == KB_F32 else _dev(lp_scale, torch.float32, "lp_scale")
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    if out is None:
        out = alloc_candidates(h, w, k_cand, planes.device)
    if workspace is None:
        workspace = alloc_workspace(n, h, w, vel.shape[0], planes.device)
    cn, ca, cv, co = out
    _check(load().kb_search(_dev(planes, planes.dtype, "planes"), code, sc_ptr, n, h, w,
                            t.ctypes.data, vel.ctypes.data, vel.shape[0], k_cand,
                            _dev(cn, torch.float32, "cand_nu"),
                            _dev(ca, torch.float32, "cand_alpha"),
                            _dev(cv, torch.int32, "cand_vel"),
                            _dev(co, torch.int16, "cand_nobs"),
                            _dev(workspace, torch.uint8, "workspace"), workspace.numel(),
                            _stream(stream)))
    return out


def search_noalloc(planes, t, vel, k_cand, out=None, stream=None, lp_scale=None):
    """kb_search_noalloc: kb_search without a workspace (the library's fixed
    device array holds the tables); same results as search()."""
    torch = _torch()
    n, h, w, two = planes.shape
    assert two == 2
    code = {torch.float32: KB_F32, torch.float16: KB_F16, torch.bfloat16: KB_BF16}[planes.dtype]
    sc_ptr = None if code == KB_F32 else _dev(lp_scale, torch.float32, "lp_scale")
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    if out is None:
        out = alloc_candidates(h, w, k_cand, planes.device)
    cn, ca, cv, co = out
    _check(load().kb_search_noalloc(_dev(planes, planes.dtype, "planes"), code, sc_ptr, n, h, w,
                                    t.ctypes.data, vel.ctypes.data, vel.shape[0], k_cand,
                                    _dev(cn, torch.float32, "cand_nu"),
                                    _dev(ca, torch.float32, "cand_alpha"),
                                    _dev(cv, torch.int32, "cand_vel"),
                                    _dev(co, torch.int16, "cand_nobs"), _stream(stream)))
    return out


def topk(cand, k, n_img, out=None, stream=None, rescore=None):
    """kb_topk: rank-ordered (nu, alpha, vel, nobs) [H][W][k].

    rescore=(planes_f32, t, vel, workspace) first recomputes every candidate
    from the float32 planes (after a 16-bit search)."""
    torch = _torch()
    cn, ca, cv, co = cand
    h, w, kc = cn.shape
    if out is None:
        out = alloc_candidates(h, w, k, cn.device)
    nu, al, vi, no = out
    pf = tp = vp = wsp = None
    nv = wsb = 0
    if rescore is not None:
        pf32, t, vel, ws = rescore
        t = _host_f64(t)
        vel = _host_f64(vel, 2)
        if ws is None:
            ws = alloc_workspace(n_img, h, w, vel.shape[0], cn.device)
        pf = _dev(pf32, torch.float32, "psi_phi_f32")
        tp, vp, nv = t.ctypes.data, vel.ctypes.data, vel.shape[0]
        wsp, wsb = _dev(ws, torch.uint8, "workspace"), ws.numel()
    _check(load().kb_topk(pf, n_img, h, w, tp, vp, nv,
                          _dev(cn, torch.float32, "cand_nu"), _dev(ca, torch.float32, "cand_alpha"),
                          _dev(cv, torch.int32, "cand_vel"), _dev(co, torch.int16, "cand_nobs"),
                          kc, k, _dev(nu, torch.float32, "nu"), _dev(al, torch.float32, "alpha"),
                          _dev(vi, torch.int32, "vel"), _dev(no, torch.int16, "nobs"), wsp, wsb,
                          _stream(stream)))
    return out


def lightcurve_filter(planes, t, vel, cand_vel, sigma_cut=5.0, q=0.0, out=None,
                      workspace=None, stream=None, rejected=False):
    """kb_lightcurve_filter: (nu, alpha, nobs) [H][W][k] refit after dropping
    outlying observations from each candidate's light curve, plus the uint64
    rejection masks (as int64) when rejected=True."""
    torch = _torch()
    n, h, w, _ = planes.shape
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    k = cand_vel.shape[-1]
    dev = planes.device
    if out is None:
        out = (torch.empty((h, w, k), dtype=torch.float32, device=dev),
               torch.empty((h, w, k), dtype=torch.float32, device=dev),
               torch.empty((h, w, k), dtype=torch.int16, device=dev))
    nu, al, no = out
    rej = torch.empty((h, w, k), dtype=torch.int64, device=dev) if rejected else None
    if workspace is None:
        workspace = alloc_workspace(n, h, w, vel.shape[0], dev)
    _check(load().kb_lightcurve_filter(
        _dev(planes, torch.float32, "psi_phi"), n, h, w, t.ctypes.data, vel.ctypes.data,
        vel.shape[0], _dev(cand_vel, torch.int32, "cand_vel"), k, float(sigma_cut), float(q),
        _dev(nu, torch.float32, "nu"), _dev(al, torch.float32, "alpha"),
        _dev(no, torch.int16, "nobs"), None if rej is None else _dev(rej, torch.int64, "rejected"),
        _dev(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))
    return (nu, al, no, rej) if rejected else (nu, al, no)


# Layout of the C struct kb_hit (24 bytes).
HIT_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("vel", "<i4"), ("nu", "<f4"),
                      ("alpha", "<f4"), ("nobs", "<i2"), ("reserved", "<i2")])


def alloc_hits(max_hits, device):
    """Device storage for max_hits kb_hit records (int32 [max_hits][6])."""
    torch = _torch()
    return torch.empty((max(int(max_hits), 1), 6), dtype=torch.int32, device=device)


def hits_to_numpy(hits, n):
    """The first n records of a hit list as a structured numpy array."""
    n = int(n)
    raw = hits[:n].contiguous().cpu().numpy()
    return raw.view(HIT_DTYPE).reshape(n)


def search_threshold(planes, t, vel, nu_min, hits, workspace=None, stream=None):
    """kb_search_threshold: appends every trajectory with nu >= nu_min to
    `hits` (from alloc_hits); returns the device counter (int64 [1]) holding
    the total number of such trajectories."""
    torch = _torch()
    n, h, w, _ = planes.shape
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    count = torch.empty(1, dtype=torch.int64, device=planes.device)
    if workspace is None:
        workspace = alloc_workspace(n, h, w, vel.shape[0], planes.device)
    _check(load().kb_search_threshold(
        _dev(planes, torch.float32, "psi_phi"), n, h, w, t.ctypes.data, vel.ctypes.data,
        vel.shape[0], float(nu_min), _dev(hits, torch.int32, "hits"), hits.shape[0],
        _dev(count, torch.int64, "n_hits"), _dev(workspace, torch.uint8, "workspace"),
        workspace.numel(), _stream(stream)))
    return count


def cluster_hits(hits, n_hits, vel, s, eps, workspace=None, stream=None):
    """kb_cluster_hits over the first n_hits records: int32 [n_hits] index of
    each hit's group representative."""
    torch = _torch()
    vel = _host_f64(vel, 2)
    n_hits = int(n_hits)
    rep = torch.empty(max(n_hits, 1), dtype=torch.int32, device=hits.device)
    if workspace is None:
        nb = load().kb_cluster_workspace_bytes(n_hits, vel.shape[0])
        workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=hits.device)
    _check(load().kb_cluster_hits(_dev(hits, torch.int32, "hits"), n_hits, vel.ctypes.data,
                                  vel.shape[0], float(s), float(eps),
                                  _dev(rep, torch.int32, "rep"),
                                  _dev(workspace, torch.uint8, "workspace"), workspace.numel(),
                                  _stream(stream)))
    return rep[:n_hits]


def stamps(img, var, mask, t, vel, cand, n_cand, radius, max_offset, max_m11, m2_min, m2_max,
           drop=None, want_stamps=True, workspace=None, stream=None):
    """kb_stamps over the first n_cand records of `cand` (kb_hit list):
    returns (pass uint8 [n], moments float64 [n][6], stamps float32
    [n][2R+1][2R+1] or None)."""
    torch = _torch()
    n, h, w = img.shape
    t = _host_f64(t)
    vel = _host_f64(vel, 2)
    n_cand = int(n_cand)
    dev = img.device
    side = 2 * int(radius) + 1
    ok = torch.empty(max(n_cand, 1), dtype=torch.uint8, device=dev)
    mom = torch.empty((max(n_cand, 1), 6), dtype=torch.float64, device=dev)
    st = (torch.empty((max(n_cand, 1), side, side), dtype=torch.float32, device=dev)
          if want_stamps else None)
    if workspace is None:
        workspace = alloc_workspace(n, h, w, vel.shape[0], dev)
    _check(load().kb_stamps(
        _dev(img, torch.float32, "img"), _dev(var, torch.float32, "var"),
        None if mask is None else _dev(mask, torch.uint8, "mask"), n, h, w, t.ctypes.data,
        vel.ctypes.data, vel.shape[0], _dev(cand, torch.int32, "cand"),
        None if drop is None else _dev(drop, torch.int64, "drop"), n_cand, int(radius),
        float(max_offset), float(max_m11), float(m2_min), float(m2_max),
        None if st is None else _dev(st, torch.float32, "stamps"),
        _dev(mom, torch.float64, "moments"), _dev(ok, torch.uint8, "pass"),
        _dev(workspace, torch.uint8, "workspace"), workspace.numel(), _stream(stream)))
    return ok[:n_cand], mom[:n_cand], (None if st is None else st[:n_cand])


def _job_array(jobs):
    """jobs: list of dicts with planes, t, vel, out (4 tensors) and optional lp_scale."""
    torch = _torch()
    arr = (KbJob * len(jobs))()
    keep = []
    for q, jb in enumerate(jobs):
        planes = jb["planes"]
        n, h, w, _ = planes.shape
        t = _host_f64(jb["t"])
        vel = _host_f64(jb["vel"], 2)
        keep += [t, vel]
        cn, ca, cv, co = jb["out"]
        sc = jb.get("lp_scale")
        arr[q] = KbJob(_dev(planes, planes.dtype, "planes"),
                       None if sc is None else _dev(sc, torch.float32, "lp_scale"),
                       n, h, w, t.ctypes.data, vel.ctypes.data, vel.shape[0],
                       _dev(cn, torch.float32, "cand_nu"), _dev(ca, torch.float32, "cand_alpha"),
                       _dev(cv, torch.int32, "cand_vel"), _dev(co, torch.int16, "cand_nobs"))
    return arr, keep


def search_batch_workspace_bytes(jobs) -> int:
    arr, keep = _job_array(jobs)
    return int(load().kb_search_batch_workspace_bytes(ctypes.addressof(arr), len(jobs)))


def search_batch(jobs, k_cand, workspace=None, stream=None):
    """kb_search_batch over several stacks sharing one plane dtype and k_cand.

    jobs: list of dicts(planes=[N][H][W][2] tensor, t, vel, out=(nu, alpha, vel, nobs)
    tensors [H][W][k_cand], lp_scale=None or [N][2]).  Returns the workspace."""
    torch = _torch()
    code = {torch.float32: KB_F32, torch.float16: KB_F16,
            torch.bfloat16: KB_BF16}[jobs[0]["planes"].dtype]
    arr, keep = _job_array(jobs)
    L = load()
    nb = int(L.kb_search_batch_workspace_bytes(ctypes.addressof(arr), len(jobs)))
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=jobs[0]["planes"].device)
    _check(L.kb_search_batch(ctypes.addressof(arr), len(jobs), code, k_cand,
                             _dev(workspace, torch.uint8, "workspace"), workspace.numel(),
                             _stream(stream)))
    return workspace


def run_search(img, var, mask, t, psf, vel, k, k_cand=None, stream=None, lp=None):
    """The whole path on device inputs: planes -> search -> top-k.
    With lp="f16"/"bf16" the search reads the scaled 16-bit planes and top-k
    re-scores every candidate from the float32 planes.
    Returns (planes, (nu, alpha, vel, nobs))."""
    k_cand = k if k_cand is None else k_cand
    if lp is None:
        planes = make_psi_phi(img, var, mask, psf, stream=stream)
        cand = search(planes, t, vel, k_cand, stream=stream)
        res = topk(cand, k, img.shape[0], stream=stream)
        return planes, res
    planes, lp_planes, scale = make_psi_phi(img, var, mask, psf, stream=stream, lp=lp)
    n, h, w = img.shape
    ws = alloc_workspace(n, h, w, np.asarray(vel).reshape(-1, 2).shape[0], img.device)
    cand = search(lp_planes, t, vel, k_cand, stream=stream, lp_scale=scale, workspace=ws)
    res = topk(cand, k, img.shape[0], stream=stream, rescore=(planes, t, vel, ws))
    return planes, res
