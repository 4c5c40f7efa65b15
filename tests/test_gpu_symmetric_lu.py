"""The symmetric FP32 factorisation of MIXED EFIE levels (no pivoting, trailing
updates of the lower triangle only, fosb_opts.lu_pivoting = 0), on the s = 4
sphere of the mixed_k5 workload (N = 7680, k = 5):

* it is the factorisation kept for the Galerkin EFIE matrix (complex
  symmetric: G and the RWG pairing are symmetric in the two arguments), and its
  refined solves and first moments agree with those of the pivoted FP32
  factorisation (lu_pivoting = 1) and of the FP64 level;
* a matrix that is not symmetric, or whose leading pivot vanishes, or whose
  elimination without pivoting grows the entries past the 1e3 limit, falls back to
  partial pivoting, and the refined solves still meet the FP64 residual bound
  for that matrix."""

import pytest

import workloads

pytestmark = pytest.mark.gpu

IR_TOL = 1e-12


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    ctx = fosb.Context(0)
    w = workloads.workload("mixed_k5")
    V, F = w.meshes[w.levels.index(4)]
    m = fosb.Mesh(ctx, V, F)
    Z = fosb.assemble(ctx, m, w.k)
    print(f"[gpu] symmetric LU: s=4 sphere, N={m.n_edges}, k={w.k}", flush=True)
    return fosb, ctx, torch, w, m, Z


def _opts(fosb, piv):
    return fosb.opts_default(ir_tol=IR_TOL, ir_max_sweeps=30, lu_pivoting=piv)


def _rhs(torch, ctx, n, nrhs=4, seed=5):
    g = torch.Generator(device="cpu").manual_seed(seed)
    B = torch.randn((n, nrhs), dtype=torch.complex128, generator=g)
    return B.to(ctx.torch_device)


def _residual(torch, Z, X, B):
    """||Z X - B||_F / (||Z||_F ||X||_F) in complex128."""
    R = torch.matmul(Z, X) - B
    return float(R.norm() / (Z.norm() * X.norm()))


def test_symmetric_factorisation_matches_pivoted_and_fp64(fz):
    fosb, ctx, torch, w, m, Z = fz
    n = m.n_edges
    lv = {}
    for name, piv in (("sym", 0), ("piv", 1)):
        lv[name] = fosb.Level(ctx, m, w.k, Z, fosb.MIXED, w.dirs, w.pols, "radial", _opts(fosb, piv))
    Z64 = Z.clone()
    lv["fp64"] = fosb.Level(ctx, m, w.k, Z64, fosb.FP64, w.dirs, w.pols, "radial", _opts(fosb, 0))
    assert lv["sym"].factorization() == fosb.FACTOR_SYM
    assert lv["piv"].factorization() == fosb.FACTOR_LU
    assert lv["fp64"].factorization() == fosb.FACTOR_LU
    B = _rhs(torch, ctx, n)
    X, sweeps = {}, {}
    for name, l in lv.items():
        st = fosb.Stats()
        X[name] = l.solve(B.clone(), st)
        sweeps[name] = st.ir_sweeps
    rel = {name: float((X[name] - X["fp64"]).norm() / X["fp64"].norm()) for name in ("sym", "piv")}
    res = {name: _residual(torch, Z, X[name], B) for name in X}
    print(f"[gpu]   refinement sweeps {sweeps}, vs FP64 {rel}, residuals {res}", flush=True)
    assert rel["sym"] < 1e-10 and rel["piv"] < 1e-10
    assert res["sym"] < 1e-13 and res["piv"] < 1e-13
    # the FP32 factors are about as good: at most one more sweep to the same tolerance
    assert sweeps["sym"] <= sweeps["piv"] + 1
    for d in range(len(w.dirs)):
        u = {name: lv[name].first_moment(d) for name in lv}
        e = float((u["sym"] - u["fp64"]).norm() / u["fp64"].norm())
        assert e < 1e-10, (d, e)
    for l in lv.values():
        l.close()


def _perturbed_level(fosb, ctx, torch, w, m, Zp):
    lv = fosb.Level(ctx, m, w.k, Zp, fosb.MIXED, w.dirs, w.pols, "radial", _opts(fosb, 0))
    B = _rhs(torch, ctx, m.n_edges, seed=7)
    X = lv.solve(B.clone())
    res = _residual(torch, Zp, X, B)
    kind = lv.factorization()
    lv.close()
    return kind, res


def test_fallback_on_asymmetry(fz):
    fosb, ctx, torch, w, m, Z = fz
    Zp = Z.clone()
    zmax = float(Z.abs().max())
    Zp[0, 1] += 1e-3 * zmax      # defect 1e-3 max|Z|, above the 1e-5 limit
    kind, res = _perturbed_level(fosb, ctx, torch, w, m, Zp)
    print(f"[gpu]   asymmetric: factorisation {kind}, residual {res:.2e}", flush=True)
    assert kind == fosb.FACTOR_LU and res < 1e-13


def test_fallback_on_zero_pivot(fz):
    fosb, ctx, torch, w, m, Z = fz
    Zp = Z.clone()
    Zp[0, 0] = 0.0               # still symmetric; the first pivot vanishes exactly
    kind, res = _perturbed_level(fosb, ctx, torch, w, m, Zp)
    print(f"[gpu]   zero pivot: factorisation {kind}, residual {res:.2e}", flush=True)
    assert kind == fosb.FACTOR_LU and res < 1e-13


def test_fallback_on_growth(fz):
    fosb, ctx, torch, w, m, Z = fz
    Zp = Z.clone()
    zmax = float(Z.abs().max())
    Zp[0, 0] = 1e-7 * zmax       # tiny leading pivot, with a coupling of max|Z| to unknown 1
    Zp[0, 1] = zmax
    Zp[1, 0] = zmax              # still symmetric
    # row 1 of U is final after the first elimination step: U11 = Z11 - Z10 Z01 / Z00
    u11 = complex(Zp[1, 1] - Zp[1, 0] * Zp[0, 1] / Zp[0, 0])
    growth_bound = abs(u11) / float(Zp.abs().max())
    assert growth_bound > 1e4
    kind, res = _perturbed_level(fosb, ctx, torch, w, m, Zp)
    print(f"[gpu]   growth >= {growth_bound:.1e}: factorisation {kind}, residual {res:.2e}", flush=True)
    assert kind == fosb.FACTOR_LU and res < 1e-13


def test_narrow_solves_match_wide_solves(fz):
    """Refined solves with 1..4 right-hand sides apply the factors' blocks as
    matrix-vector products (the narrow kernel); with 5 as GEMMs.  Both meet the
    same refinement tolerance, so the same columns agree to it, and each has an
    FP64-level residual."""
    fosb, ctx, torch, w, m, Z = fz
    lv = fosb.Level(ctx, m, w.k, Z, fosb.MIXED, w.dirs, w.pols, "radial", _opts(fosb, 0))
    B = _rhs(torch, ctx, m.n_edges, nrhs=5, seed=11)
    wide = lv.solve(B.clone())
    for k in (1, 2, 3, 4):
        narrow = lv.solve(B[:, :k].contiguous().clone())
        rel = float((narrow - wide[:, :k]).norm() / wide[:, :k].norm())
        res = _residual(torch, Z, narrow, B[:, :k].contiguous())
        print(f"[gpu]   {k} right-hand sides: vs the 5-column solve {rel:.2e}, residual {res:.2e}", flush=True)
        assert rel < 1e-10 and res < 1e-13
    lv.close()
