"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/fosb.h, and its host-only entry points
(mesh validation, CT index set, defaults) behave as documented."""

import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fosb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fosb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("fosb_assemble", "fosb_rhs_correlation", "fosb_correlation", "fosb_far_field_moments",
              "fosb_two_sided_solve", "fosb_level_create", "fosb_mesh_create", "fosb_ct_pairs"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2308_01457_amd import fosb
    L = fosb.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert name in fosb._SIGS, f"binding does not marshal {name}"


def test_ct_pairs_match_oracle():
    from oracle import uq
    from paper_2308_01457_amd import fosb
    for L0, L in ((1, 3), (2, 5), (0, 2), (3, 6), (4, 4), (0, 7)):
        assert fosb.ct_pairs(L0, L) == [tuple(p) for p in uq.ct_pairs(L0, L)]


def test_ct_pairs_rejects_bad_range():
    from paper_2308_01457_amd import fosb
    with pytest.raises(fosb.FosbError) as e:
        fosb.ct_pairs(3, 2)
    assert e.value.name == "E_INVALID"


def test_opts_default():
    from paper_2308_01457_amd import fosb
    o = fosb.opts_default()
    assert o.n_gauss_singular == 5 and o.ir_max_sweeps == 10 and o.ir_tol == 1e-10


def test_mesh_validate_counts_edges():
    from paper_2308_01457_amd import fosb
    for s in range(4):
        V, F = workloads.icosphere(s)
        assert fosb.mesh_validate(V, F) == 30 * 4 ** s
    V, F = workloads.geodesic_sphere(5)
    assert fosb.mesh_validate(V, F) == 30 * 25


@pytest.mark.parametrize("case", ["open", "nonmanifold", "flipped_one", "inward", "degenerate", "nan",
                                  "index_range"])
def test_mesh_validate_rejects_like_the_oracle(case):
    from oracle import mesh as omesh
    from paper_2308_01457_amd import fosb
    V, F = workloads.icosphere(1)
    V = V.copy()
    F = F.copy()
    if case == "open":
        F = F[1:]
    elif case == "nonmanifold":
        F = np.vstack([F, F[:1]])
    elif case == "flipped_one":
        F[3] = F[3][[0, 2, 1]]
    elif case == "inward":
        F = F[:, [0, 2, 1]]
    elif case == "degenerate":
        V[F[0, 1]] = V[F[0, 0]] + 1e-18
    elif case == "nan":
        V[0, 0] = np.nan
    elif case == "index_range":
        F[0, 0] = V.shape[0]
    with pytest.raises(fosb.FosbError) as e:
        fosb.mesh_validate(V, F)
    assert e.value.name == "E_INVALID"
    with pytest.raises(omesh.MeshError):
        omesh.build(V, F)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2308_01457_amd import fosb
    monkeypatch.setattr(fosb, "_lib", None)
    monkeypatch.setattr(fosb, "LIB_PATH", str(tmp_path / "libfosb.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        fosb.lib()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stdout
