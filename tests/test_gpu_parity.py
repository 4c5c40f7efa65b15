"""GPU path vs the FP64 oracle on the plain FP64 workload (unit icosphere
s=1..3, k=1, d=e_z, p=e_x, radial Gaussian covariance sigma=0.01, ell=0.5,
L0=1, L=3, 181 angles in the xz-plane), plus solver properties.

Tolerances: the FP64 path reproduces the oracle to rounding (relative 1e-10
allowed on blocks and variance, 1e-12 on the matrix); the mixed path must meet
its 1e-5 bound on every block and on the variance (it refines to ~1e-10)."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K1 = 1.0
SIG, ELL = 0.01, 0.5


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    ctx = fosb.Context(0)
    return fosb, ctx, torch


@pytest.fixture(scope="module")
def gpu_levels(fz):
    fosb, ctx, torch = fz
    out = {}
    for s in (1, 2, 3):
        V, F = workloads.icosphere(s)
        print(f"[gpu] assemble + factor icosphere s={s}", flush=True)
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, K1)
        Zc = Z.clone()
        lv = fosb.Level(ctx, m, K1, Z, fosb.FP64)
        out[s] = (m, Zc, lv)
    torch.cuda.synchronize()
    return out


def test_assemble_matches_oracle(fz, gpu_levels, oracle_levels):
    for s in (1, 2, 3):
        Zg = gpu_levels[s][1].cpu().numpy()
        Zo = oracle_levels(s).Z
        err = np.abs(Zg - Zo).max() / np.abs(Zo).max()
        print(f"[gpu] Z s={s} max rel err {err:.2e}", flush=True)
        assert err < 1e-12


def test_assemble_other_wavenumber_and_gauss_order(fz):
    fosb, ctx, torch = fz
    from oracle import efie, mesh
    V, F = workloads.icosphere(2)
    m = fosb.Mesh(ctx, V, F)
    for k, ng in ((5.0, 5), (2.5, 3)):
        print(f"[gpu] assemble s=2 k={k} n_G={ng}", flush=True)
        Zg = fosb.assemble(ctx, m, k, fosb.opts_default(n_gauss_singular=ng)).cpu().numpy()
        Zo = efie.assemble(mesh.build(V, F), k, n_gauss=ng)
        assert np.abs(Zg - Zo).max() / np.abs(Zo).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_level_solve_blocked_lookahead_sizes(fz, precision):
    """Sizes that take the blocked, two-stream LU: N = 2430 (geodesic sphere
    nu = 9: neither a multiple of the 32-column panel nor of the 256-column
    block) and N = 7680 (icosphere s = 4); backward error of X = Z^{-1} B and
    of X = Z^{-H} B, measured on the GPU against the kept matrix."""
    fosb, ctx, torch = fz
    rng = np.random.default_rng(8)
    for name, (V, F), nrhs in (("nu9", workloads.geodesic_sphere(9), 5), ("s4", workloads.icosphere(4), 3)):
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, K1)
        Zc = Z.clone()
        prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
        print(f"[gpu] blocked LU {precision} {name} N={m.n_edges}", flush=True)
        lv = fosb.Level(ctx, m, K1, Z, prec, opts=fosb.opts_default(ir_tol=1e-13))  # refine to the FP64 floor
        B = torch.tensor(rng.standard_normal((m.n_edges, nrhs)) + 1j * rng.standard_normal((m.n_edges, nrhs)),
                         device=ctx.torch_device)
        nz = torch.linalg.matrix_norm(Zc).item()   # Frobenius (>= the 2-norm)
        X = lv.solve(B.clone())
        bwd = (torch.linalg.matrix_norm(Zc @ X - B) / (nz * torch.linalg.matrix_norm(X))).item()
        Xa = lv.solve_adjoint(B.clone())
        bwa = (torch.linalg.matrix_norm(Zc.conj().T.contiguous() @ Xa - B) / (nz * torch.linalg.matrix_norm(Xa))).item()
        print(f"[gpu]   backward error {bwd:.2e}, adjoint {bwa:.2e}", flush=True)
        assert bwd < 1e-14 and bwa < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_level_solve_backward_error(fz, precision):
    """X = Z^{-1} B on ragged sizes (N = 120, 480, 1920; nrhs 1, 7, 33): small
    backward error and agreement with LAPACK on the same matrix."""
    fosb, ctx, torch = fz
    rng = np.random.default_rng(5)
    for s, nrhs in ((1, 7), (2, 33), (3, 1)):
        V, F = workloads.icosphere(s)
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, K1)
        Zc = Z.clone().cpu().numpy()
        prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
        print(f"[gpu] solve {precision} s={s} nrhs={nrhs}", flush=True)
        lv = fosb.Level(ctx, m, K1, Z, prec, opts=fosb.opts_default(ir_tol=1e-13))  # refine to the FP64 floor
        B = rng.standard_normal((m.n_edges, nrhs)) + 1j * rng.standard_normal((m.n_edges, nrhs))
        Bt = torch.tensor(B, device=ctx.torch_device)
        st = fosb.Stats()
        X = lv.solve(Bt, st).cpu().numpy()
        bwd = np.linalg.norm(Zc @ X - B) / (np.linalg.norm(Zc, 2) * np.linalg.norm(X))
        ref = np.linalg.solve(Zc, B)
        print(f"[gpu]   backward {bwd:.2e} forward {_rel(X, ref):.2e} sweeps {st.ir_sweeps}", flush=True)
        assert bwd < 1e-14
        assert _rel(X, ref) < 1e-9


def test_first_moment_matches_oracle(fz, gpu_levels, oracle_levels):
    for s in (1, 2, 3):
        u = gpu_levels[s][2].first_moment().cpu().numpy()
        assert _rel(u, oracle_levels(s).u) < 1e-10


def test_rhs_correlation_matches_oracle(fz, gpu_levels, oracle_levels):
    fosb, ctx, torch = fz
    from oracle import uq
    cov = fosb.make_cov("gaussian", SIG, ELL)
    for a, b in ((3, 1), (2, 2), (2, 1), (1, 3)):
        Cg = fosb.rhs_correlation(ctx, gpu_levels[a][2], gpu_levels[b][2], cov).cpu().numpy()
        Co = uq.rhs_correlation(oracle_levels(a), oracle_levels(b), "gaussian", SIG, ELL)
        print(f"[gpu] C({a},{b}) rel err {_rel(Cg, Co):.2e}", flush=True)
        assert _rel(Cg, Co) < 1e-10


def test_ct_blocks_and_variance_match_oracle_fp64(fz, gpu_levels, oracle_levels):
    fosb, ctx, torch = fz
    from oracle import uq
    xh = workloads.angles_xz(181)
    levels = [gpu_levels[s][2] for s in (1, 2, 3)]
    cov = fosb.make_cov("gaussian", SIG, ELL)
    print("[gpu] CT correlation L0=1 L=3 fp64", flush=True)
    blocks = fosb.correlation(ctx, levels, 1, 3, cov)
    var = fosb.far_field_moments(ctx, levels, 1, 3, blocks, xh).cpu().numpy()
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    Vo, per, oblocks, _, _ = uq.second_moment(None, K1, 1, 3, "gaussian", SIG, ELL, xh, levels=olv)
    for (a, b, sg, mu), blk in zip(fosb.ct_pairs(1, 3), blocks):
        e = _rel(blk.cpu().numpy(), oblocks[(a, b)])
        print(f"[gpu] Sigma({a},{b}) rel err {e:.2e}", flush=True)
        assert e < 1e-10
    print(f"[gpu] variance rel err {_rel(var, Vo):.2e}", flush=True)
    assert _rel(var, Vo) < 1e-10


def test_ct_variance_mixed_precision(fz, oracle_levels):
    fosb, ctx, torch = fz
    from oracle import uq
    xh = workloads.angles_xz(181)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    print("[gpu] full pipeline mixed precision", flush=True)
    res = fosb.run_pipeline(ctx, [workloads.icosphere(s) for s in (1, 2, 3)], K1, 1, 3, cov, xh, fosb.MIXED)
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    Vo, per, oblocks, _, _ = uq.second_moment(None, K1, 1, 3, "gaussian", SIG, ELL, xh, levels=olv)
    for (a, b, sg, mu), blk in zip(fosb.ct_pairs(1, 3), res.blocks):
        assert _rel(blk.cpu().numpy(), oblocks[(a, b)]) < 1e-5
    e = _rel(res.var.cpu().numpy(), Vo)
    print(f"[gpu] mixed variance rel err {e:.2e}, sweeps {res.stats.ir_sweeps}", flush=True)
    assert e < 1e-5
