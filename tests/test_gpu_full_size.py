"""GPU path at the benchmark's full size (workload mixed_k5: unit icosphere
s = 2..5, N up to 30720, k = 5, radial Gaussian covariance (0.01, 0.5),
L0 = 2, L = 5, 181 angles), in the launch configuration bench.py times.

* Sampled EFIE entries of the s = 5 matrix (random pairs plus every touching
  kind) against the oracle's entry-by-entry integration.
* Every CT pair's far-field variance contribution, sampled Sigma and C entries,
  sampled first moments and each level's first-moment far field against
  tests/golden/mixed_k5_oracle.json, which make_mixed_k5_golden.py wrote from
  the oracle alone.  FP64 path: 1e-9; mixed path (bench tolerance: refined
  solves to an estimated 1e-7): 1e-6 on the variance, 1e-5 on sampled entries (C is
  built from the first moments, so it carries their accuracy).
* The CT variance against the mesh-free spectral Mie shape derivative
  (tests/golden/mie_shape_oracle.json): within 0.2%, the discretisation and
  combination-technique error at L = 5.
* Properties at full size: the two-sided backward error of the (5,2) block
  and the Hermitian symmetry of C(3,3)."""

import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "mixed_k5_oracle.json")
BENCH_IR_TOL = 1e-7   # bench.py's default target error of the refined solves


def _c(d):
    return np.asarray(d["re"]) + 1j * np.asarray(d["im"])


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def test_sampled_entries_top_level(fz):
    fosb, ctx, torch = fz
    from oracle import efie, mesh
    w = workloads.workload("mixed_k5")
    V, F = w.meshes[-1]
    om = mesh.build(V, F)
    rng = np.random.default_rng(99)
    rows = list(rng.integers(0, om.ne, 96))
    cols = list(rng.integers(0, om.ne, 96))
    # touching kinds: diagonal, RWGs sharing a triangle, RWGs on adjacent triangles
    for e in rng.integers(0, om.ne, 16):
        t = om.edge_tri[e, 0]
        rows += [e, e]
        cols += [e, om.tri_edge[t, (list(om.tri_edge[t]).index(e) + 1) % 3]]
        t2 = om.edge_tri[e, 1]
        rows.append(e)
        cols.append(om.tri_edge[t2, (list(om.tri_edge[t2]).index(e) + 1) % 3])
    rows, cols = np.array(rows), np.array(cols)
    print(f"[gpu] full-size assembly s=5 k={w.k}: {len(rows)} sampled entries", flush=True)
    m = fosb.Mesh(ctx, V, F)
    Z = fosb.assemble(ctx, m, w.k)
    idx = torch.tensor(rows * om.ne + cols, device=ctx.torch_device)
    zg = Z.view(-1)[idx].cpu().numpy()
    zmax = float(Z.abs().max().item())
    del Z
    zo = efie.entries(om, w.k, rows, cols)
    err = np.abs(zg - zo).max() / zmax
    print(f"[gpu]   max |Z_gpu - Z_oracle| / max|Z| = {err:.2e}", flush=True)
    assert err < 1e-12


def _run(fosb, ctx, torch, precision):
    w = workloads.workload("mixed_k5")
    opts = fosb.opts_default(ir_tol=BENCH_IR_TOL if precision == fosb.MIXED else 1e-10, ir_max_sweeps=10)
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    meshes, levels = [], []
    for s, (V, F) in zip(w.levels, w.meshes):
        m = fosb.Mesh(ctx, V, F)
        Z = fosb.assemble(ctx, m, w.k, opts)
        lv = fosb.Level(ctx, m, w.k, Z, precision, w.dirs, w.pols, "radial", opts)
        meshes.append(m)
        levels.append(lv)
        print(f"[gpu]   level s={s} N={m.n_edges} factored", flush=True)
    st = fosb.Stats()
    blocks = fosb.correlation(ctx, levels, w.L0, w.L, cov, 0, stats=st)
    var = fosb.far_field_moments(ctx, levels, w.L0, w.L, blocks, w.angles).cpu().numpy()
    return w, cov, meshes, levels, blocks, var, st


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_against_oracle_golden(fz, golden, precision):
    fosb, ctx, torch = fz
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    print(f"[gpu] full-size pipeline mixed_k5 {precision}", flush=True)
    w, cov, meshes, levels, blocks, var, st = _run(fosb, ctx, torch, prec)
    tol_v, tol_e = (1e-9, 1e-9) if precision == "fp64" else (1e-6, 1e-5)
    xh = w.angles
    for i, s in enumerate(w.levels):
        g = golden["per_level"][str(s)]
        u = levels[i].first_moment().cpu().numpy()
        e_u = _rel(u[np.array(g["u_idx"])], _c(g["u"]))
        FF = fosb.far_field_matrix(ctx, levels[i], xh)
        Fg = (FF @ levels[i].first_moment().view(-1, 1)).view(3, -1).cpu().numpy().T
        e_f = _rel(Fg, _c(g["far_field"]))
        print(f"[gpu]   s={s}: first moment {e_u:.2e}, far field {e_f:.2e}", flush=True)
        assert e_u < tol_e and e_f < tol_e
    for (l1, l2, sg, mu), blk, gp in zip(fosb.ct_pairs(w.L0, w.L), blocks, golden["pairs"]):
        assert (gp["l1"], gp["l2"]) == (l1, l2)
        a, b = levels[l1 - w.L0], levels[l2 - w.L0]
        FF1 = fosb.far_field_matrix(ctx, a, xh)
        FF2 = fosb.far_field_matrix(ctx, b, xh)
        Vp = torch.real(((FF1 @ blk) * FF2.conj()).sum(dim=1)).view(3, -1).cpu().numpy()
        e_v = _rel(Vp, np.asarray(gp["pair_variance"]))
        si = np.asarray(gp["Sigma_idx"])
        sg_gpu = blk[torch.tensor(si[0], device=ctx.torch_device),
                     torch.tensor(si[1], device=ctx.torch_device)].cpu().numpy()
        e_s = _rel(sg_gpu, _c(gp["Sigma"]))
        ci = np.asarray(gp["C_idx"])
        Cg = fosb.rhs_correlation(ctx, a, b, cov)
        c_gpu = Cg[torch.tensor(ci[0], device=ctx.torch_device),
                   torch.tensor(ci[1], device=ctx.torch_device)].cpu().numpy()
        del Cg
        e_c = _rel(c_gpu, _c(gp["C"]))
        print(f"[gpu]   pair ({l1},{l2}): variance {e_v:.2e}, Sigma samples {e_s:.2e}, C samples {e_c:.2e}",
              flush=True)
        assert e_v < tol_v and e_s < tol_e and e_c < tol_e   # C inherits the first moments' accuracy
    e = _rel(var, np.asarray(golden["variance"]))
    print(f"[gpu]   CT variance {e:.2e} (refinement sweeps {st.ir_sweeps})", flush=True)
    assert e < tol_v
    # the mesh-free spectral Mie value of the same variance (discretisation + CT error at L = 5)
    with open(os.path.join(HERE, "golden", "mie_shape_oracle.json")) as f:
        mie = np.asarray(json.load(f)["variance"]["5.0"])
    e_m = _rel(var, mie)
    print(f"[gpu]   CT variance vs the spectral Mie shape derivative {e_m:.2e}", flush=True)
    assert e_m < 2e-3


def test_full_size_properties(fz):
    """Two-sided backward error of the (5,2) block and C(3,3) = C(3,3)^H,
    on the mixed path with the bench tolerance (the caller's Z stays
    unfactored, so the residual is formed against the assembled matrices)."""
    fosb, ctx, torch = fz
    w = workloads.workload("mixed_k5")
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    opts = fosb.opts_default(ir_tol=BENCH_IR_TOL)
    Z, lv = {}, {}
    for s, (V, F) in zip(w.levels, w.meshes):
        if s not in (2, 3, 5):
            continue
        m = fosb.Mesh(ctx, V, F)
        Z[s] = fosb.assemble(ctx, m, w.k, opts)
        lv[s] = fosb.Level(ctx, m, w.k, Z[s], fosb.MIXED, w.dirs, w.pols, "radial", opts)
    print("[gpu] full-size properties: (5,2) two-sided backward error, C(3,3) Hermitian", flush=True)
    C = fosb.rhs_correlation(ctx, lv[5], lv[2], cov)
    S = fosb.two_sided_solve(ctx, lv[5], lv[2], C.clone())
    R = Z[5] @ S @ Z[2].conj().T.contiguous() - C
    nz5 = torch.linalg.matrix_norm(Z[5]).item()
    nz2 = torch.linalg.matrix_norm(Z[2]).item()
    bwd = torch.linalg.matrix_norm(R).item() / (nz5 * torch.linalg.matrix_norm(S).item() * nz2)
    print(f"[gpu]   (5,2): ||Z5 S Z2^H - C||_F / (||Z5||_F ||S||_F ||Z2||_F) = {bwd:.2e}", flush=True)
    assert bwd < 1e-7      # refined to an estimated relative error of 1e-7
    C33 = fosb.rhs_correlation(ctx, lv[3], lv[3], cov)
    herm = (torch.linalg.matrix_norm(C33 - C33.conj().T) / torch.linalg.matrix_norm(C33)).item()
    print(f"[gpu]   C(3,3) Hermitian defect {herm:.2e}", flush=True)
    assert herm < 1e-13
