"""fosb_far_field_moments_noalloc (work memory in the library's per-GPU
device array, no allocation) against fosb_far_field_moments on the same
levels and Sigma blocks, through the C ABI:
* the plain workload's ladder (s = 1..3, k = 1) with 181 angles, then the
  differentiated workload's ladder (s = 1..4, k = 3) with 181 angles, which
  the array takes in several angle chunks, then a smaller input (s = 1..2,
  37 angles) on the same array: variance and mean field to 1e-12 (the only
  difference is the summation order of split-K GEMM products);
* no device allocation is made by any of these calls."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SIG, ELL = 0.01, 0.5


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def _ladder(fosb, ctx, levels_s, k, precision, cov, L0, L):
    lv = []
    for s in levels_s:
        m = fosb.Mesh(ctx, *workloads.icosphere(s))
        lv.append(fosb.Level(ctx, m, k, fosb.assemble(ctx, m, k), precision))
    return lv, fosb.correlation(ctx, lv, L0, L, cov)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_far_field_moments(fz, precision):
    fosb, ctx, torch = fz
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    cov = fosb.make_cov("gaussian", SIG, ELL)
    cases = [((1, 2, 3), 1.0, 181), ((1, 2, 3, 4), 3.0, 181), ((1, 2), 1.0, 37)]
    for levels_s, k, n_a in cases:
        L0, L = levels_s[0], levels_s[-1]
        xh = workloads.angles_xz(n_a)
        lv, blocks = _ladder(fosb, ctx, levels_s, k, prec, cov, L0, L)
        ref, ref_mean = fosb.far_field_moments(ctx, lv, L0, L, blocks, xh, with_mean=True)
        ref, ref_mean = ref.cpu().numpy().ravel(), ref_mean.cpu().numpy().ravel()
        var = torch.full((3 * n_a,), np.nan, dtype=torch.float64, device=ctx.torch_device)
        mean = torch.full((3 * n_a,), np.nan, dtype=torch.complex128, device=ctx.torch_device)
        before = ctx.memory()["n_device_allocs"]
        print(f"[gpu] noalloc {precision} levels {levels_s} k={k} n_a={n_a}", flush=True)
        fosb.far_field_moments_noalloc(ctx, lv, L0, L, blocks, xh, var, mean=mean)
        after = ctx.memory()["n_device_allocs"]
        v, mf = var.cpu().numpy(), mean.cpu().numpy()
        ev = float(np.abs(v - ref).max() / np.abs(ref).max())
        em = float(np.abs(mf - ref_mean).max() / np.abs(ref_mean).max())
        print(f"[gpu]   variance {ev:.2e}, mean field {em:.2e}, allocations {before} -> {after}", flush=True)
        assert after == before
        assert ev < 1e-12 and em < 1e-12
