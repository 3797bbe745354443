"""Host logic of bench.py's precision-mode comparison, on CPU tensors with a
stand-in library (no GPU): recall against the float32 path, the bitwise
equality check of kept trajectories, and the pre-re-score error units."""
import types

import numpy as np
import pytest
import torch

import bench

H, W, K, KC = 8, 5, 3, 5


class _FakeLib:
    """kb_search / kb_topk stand-ins: plain top-k gives `ref`, the re-score of
    the 16-bit candidates gives `full` (float32 values of every candidate)."""

    def __init__(self, ref, full):
        self.ref, self.full = ref, full

    def search(self, planes, t, vel, k, workspace=None):
        return ("candidates", k)

    def topk(self, cand, k, n, rescore=None):
        return self.ref if rescore is None else self.full


def _torch_ns():
    return types.SimpleNamespace(
        cuda=types.SimpleNamespace(synchronize=lambda: None), float32=torch.float32,
        int32=torch.int32, arange=torch.arange, gather=torch.gather, isfinite=torch.isfinite,
        maximum=torch.maximum, equal=torch.equal)


def _lists(seed=0):
    g = torch.Generator().manual_seed(seed)
    vel = torch.stack([torch.randperm(20, generator=g)[:KC] for _ in range(H * W)])
    vel = vel.reshape(H, W, KC).int()
    nu = torch.rand(H, W, KC, generator=g) * 10 + 1.0
    order = torch.argsort(-nu, -1)
    nu, vel = torch.gather(nu, -1, order), torch.gather(vel, -1, order)
    full = (nu, nu * 0.5, vel, torch.full_like(vel, 7).short())
    ref = tuple(t[..., :K].contiguous() for t in full)
    return full, ref


def _run(full, ref, res, cand):
    return bench.precision_vs_f32(_FakeLib(ref, full), _torch_ns(), torch.zeros(2, H, W, 2),
                                  cand, tuple(res), types.SimpleNamespace(k=K, t=None, vel=None),
                                  KC, None, row_stride=2, chunk_rows=3)


def test_recall_counts_missing_float32_entries():
    full, ref = _lists()
    res = [t.clone() for t in ref]
    for f, r in zip(full, res):            # pixel (0, 0) kept its 4th candidate instead of its 3rd
        r[0, 0, K - 1] = f[0, 0, K]
    out = _run(full, ref, res, full)
    assert out["recall_vs_f32"] == pytest.approx(1 - 1 / (H * W * K), abs=1e-12)
    assert out["kept_values_bitwise_equal_f32"]
    assert out["nu_err_before_rescore"]["max"] == 0.0


def test_bitwise_check_sees_a_changed_value():
    full, ref = _lists(1)
    res = [t.clone() for t in ref]
    res[1][3, 2, 0] = torch.nextafter(res[1][3, 2, 0], torch.tensor(np.inf))
    assert not _run(full, ref, res, full)["kept_values_bitwise_equal_f32"]


def test_errors_before_rescore_in_tolerance_units():
    full, ref = _lists(2)
    # 16-bit scores 1e-3 above the float32 ones, same order
    cand = (full[0] + 1e-3, full[1], full[2], full[3])
    out = _run(full, ref, [t.clone() for t in ref], cand)
    # nu >= 1 here, so the unit is |nu|: the relative error of each value
    want = (1e-3 / full[0][::2].double()).max().item()
    assert out["nu_err_before_rescore"]["max"] == pytest.approx(want, rel=1e-4)
    assert out["nu_err_before_rescore"]["n"] == (H // 2) * W * KC
    assert out["alpha_err_before_rescore"]["max"] == 0.0


def test_cpu_baseline_and_recall_on_a_small_stack():
    """bench.cpu_baseline runs the C oracle on a block of start rows (the TIE
    it credits are the rows it computes) and recall_vs_fp64 checks lists
    against it: the oracle's own top-k in float32 recalls everything."""
    from paper_1901_02492_amd import synth
    s = synth.random_stack(501, n=5, h=48, w=40, n_vel=20, k=4, psf_size=5, vmax=6.0, tmax=1.0)
    base, rows = bench.cpu_baseline(s)
    arrays, r0, r1 = rows
    assert r0 < r1 <= 48 and arrays["vel"].shape == (r1 - r0, 40, 12)
    assert base["kind"] == "oracle" and base["value"] > 0 and base["cores"] >= 1
    assert f"{r1 - r0} full-width rows" in base["sample"]
    full = np.zeros((48, 40, 4), np.float32)
    res = [torch.from_numpy(full.copy()), torch.from_numpy(full.copy()),
           torch.from_numpy(full.astype(np.int32)), torch.from_numpy(full.astype(np.int16))]
    for t, key in zip(res, ("nu", "alpha", "vel", "nobs")):
        t[r0:r1] = torch.from_numpy(np.ascontiguousarray(arrays[key][..., :4]).astype(
            t.numpy().dtype))
    rec = bench.recall_vs_fp64(rows, res, 4)
    assert rec["value"] == 1.0 and rec["pixels"] == (r1 - r0) * 40
