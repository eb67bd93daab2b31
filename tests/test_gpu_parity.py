"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (FP64 path): kept ranks per cluster and step identical; preconditioner apply
equal to the oracle's within 1e-10 relative (max-norm); PCG iteration counts within
+-1 and the true relative residual <= 1e-12; with nothing truncated (eps = 0, or
sparsification skipped) the apply equals a dense Cholesky solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import gridgen
from oracle import spand_oracle as O
from tests.gpu_util import (gpu_apply, gpu_factor, gpu_solve, note, oracle_run, rank_mismatches)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note(request.node.nodeid)


SMALL = [
    ("lap2d_7x7_L3", lambda: gridgen.laplacian((7, 7)), 3, 1e-2, 0),
    ("lap2d_16x16_L5", lambda: gridgen.laplacian((16, 16)), 5, 1e-2, 0),
    ("lap3d_8x8x8_L5", lambda: gridgen.laplacian((8, 8, 8)), 5, 1e-2, 0),
    ("lap3d_9x7x6_L4_eps0", lambda: gridgen.laplacian((9, 7, 6)), 4, 0.0, 0),
    ("lap3d_9x7x6_L4_direct", lambda: gridgen.laplacian((9, 7, 6)), 4, 0.1, 99),
    ("var3d_10x9x8_L5", lambda: gridgen.variable_coefficient((10, 9, 8), np.random.default_rng(21), -3, 3), 5, 1e-2, 0),
    ("lap3d_13x11x9_L6_eps0.5", lambda: gridgen.laplacian((13, 11, 9)), 6, 0.5, 0),
    ("c1_lap2d_64x64_L6", lambda: gridgen.config_problem("c1")[0], 6, 1e-2, 0),
]


@pytest.mark.parametrize("name,make,levels,tol,skip", SMALL, ids=[c[0] for c in SMALL])
def test_small_parity(name, make, levels, tol, skip):
    p = make()
    b = gridgen.rhs(np.random.default_rng(100), p.n, 2)
    an, fac = oracle_run(p, levels, tol, skip)
    s = gpu_factor(p, levels, tol, skip)
    assert rank_mismatches(s, an, fac) == 0
    z_gpu = gpu_apply(s, b)
    z_ref = O.apply(fac, b)
    assert np.abs(z_gpu - z_ref).max() <= 1e-10 * np.abs(z_ref).max()
    x, it, rr, _ = gpu_solve(s, b)
    _, it_ref, rr_ref = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    assert np.all(np.abs(it - it_ref) <= 1), (it, it_ref)
    assert np.all(rr <= 1e-12), rr
    st = s.stats()
    assert st["s_top"] == fac.stats["s_top"]
    assert st["m_F"] == fac.stats["m_F"]


@pytest.mark.parametrize("shape,levels,skip,tol", [((9, 7, 6), 4, 0, 0.0), ((12, 10), 4, 99, 0.3),
                                                   ((6, 6, 6), 3, 0, 0.0)])
def test_exact_factorization_matches_dense_solve(shape, levels, skip, tol):
    p = gridgen.laplacian(shape)
    b = gridgen.rhs(np.random.default_rng(5), p.n, 3)
    s = gpu_factor(p, levels, tol, skip)
    z = gpu_apply(s, b)
    x_ref = sla.cho_solve(sla.cho_factor(p.scipy().toarray()), b)
    assert np.abs(z - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
    x, it, rr, _ = gpu_solve(s, b)
    assert np.all(it == 1) and np.all(rr < 1e-13)


@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-4])
def test_c2_laplacian_32cubed(tol):
    """3D 7-point Laplacian 32^3, 9 levels, one RHS (seed 2), PCG to 1e-12."""
    p, b, L = gridgen.config_problem("c2")
    an, fac = oracle_run(p, L, tol)
    s = gpu_factor(p, L, tol)
    mism = rank_mismatches(s, an, fac)
    x, it, rr, _ = gpu_solve(s, b)
    _, it_ref, rr_ref = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    note(f"c2 tol={tol}: iters gpu {it} oracle {it_ref}, relres {rr}, rank mismatches {mism}")
    assert np.all(np.abs(it - it_ref) <= 1)
    assert np.all(rr <= 1e-12)
    assert mism == 0
    if mism == 0:
        z = gpu_apply(s, b)
        zr = O.apply(fac, b)
        assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()


def test_multi_rhs_columns_independent():
    """8 right-hand sides solved together give each column's single-RHS result."""
    p = gridgen.laplacian((12, 11, 10))
    b = gridgen.rhs(np.random.default_rng(8), p.n, 8)
    s = gpu_factor(p, 6, 1e-2)
    X, it, rr, _ = gpu_solve(s, b)
    for c in [0, 3, 7]:
        x1, it1, rr1, _ = gpu_solve(s, b[:, c:c + 1])
        assert it1[0] == it[c]
        assert np.abs(x1[:, 0] - X[:, c]).max() <= 1e-12 * np.abs(X[:, c]).max()


def test_apply_many_rhs_matches_oracle():
    """Eleven right-hand sides (a full block of eight and a ragged block of three) through
    the tiled apply products, on a 24^3 Laplacian at 5 levels whose upper clusters span
    several 64-wide tiles with a ragged last tile.  Its interfaces take every CPQR
    register layout: one workgroup, the wide single workgroup, and several workgroups
    in each of the two multi-slab layouts, some with a column per team in LDS beside
    the register columns; the ranks and the apply (which reads the reflectors, T
    factors and W blocks they wrote) are checked against the oracle."""
    p = gridgen.laplacian((24, 24, 24))
    b = gridgen.rhs(np.random.default_rng(12), p.n, 11)
    an, fac = oracle_run(p, 5, 1e-2)
    s = gpu_factor(p, 5, 1e-2)
    assert rank_mismatches(s, an, fac) == 0
    st = s.stats()
    assert st["s_top"] > 64
    assert all(k > 0 for k in st["cpqr_interfaces"]), st["cpqr_interfaces"]
    assert st["cpqr_lds_slot_interfaces"] > 0, st
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()


def test_zero_rhs_column():
    p = gridgen.laplacian((10, 10))
    b = gridgen.rhs(np.random.default_rng(3), p.n, 3)
    b[:, 1] = 0.0
    s = gpu_factor(p, 4, 1e-2)
    x, it, rr, _ = gpu_solve(s, b)
    assert it[1] == 0 and np.all(x[:, 1] == 0.0) and rr[1] == 0.0
    assert it[0] > 0 and rr[0] <= 1e-12


def test_deterministic_fp64():
    """Two factor+solve runs give bit-identical solutions (ordered Schur reduction)."""
    p = gridgen.variable_coefficient((14, 13, 12), np.random.default_rng(4), -2, 2)
    b = gridgen.rhs(np.random.default_rng(9), p.n, 2)
    xs = []
    for _ in range(2):
        s = gpu_factor(p, 6, 1e-2)
        x, it, rr, _ = gpu_solve(s, b)
        xs.append(x)
    assert np.array_equal(xs[0], xs[1])


def test_refactor_schedule_is_bit_identical():
    """A refactorization at the same tolerance lists the multi-slab CPQR work by the
    ranks of the previous factorization, and the colour classes' multi-slab launches run
    on a second stream beside the single-slab ones: neither changes a bit of the
    factors.  The 24^3 Laplacian at 5 levels takes every CPQR layout; the apply after
    the second factorization equals the first bit for bit, with the same ranks."""
    p = gridgen.laplacian((24, 24, 24))
    b = gridgen.rhs(np.random.default_rng(13), p.n, 3)
    from paper_1901_02971_amd import Solver
    vals = torch.from_numpy(p.values).to("cuda:0")
    s = Solver.from_problem(p, 5)
    s.factor(vals, 1e-2)
    st1 = s.stats()
    assert all(k > 0 for k in st1["cpqr_interfaces"]), st1["cpqr_interfaces"]
    z1 = gpu_apply(s, b)
    s.factor(vals, 1e-2)
    st2 = s.stats()
    z2 = gpu_apply(s, b)
    assert np.array_equal(z1, z2)
    assert (st1["s_top"], st1["m_F"]) == (st2["s_top"], st2["m_F"])
    s.close()


@pytest.mark.parametrize("shape,levels", [((32, 32, 32), 9), ((40, 40, 40), 8)])
def test_one_launch_cpqr_steps_match_oracle(shape, levels):
    """Steps whose CPQR work lies mostly in multi-slab interfaces run all colour classes
    in one cooperative launch, each interface waiting on device counters for its
    neighbours of earlier classes (and reading their write-back and ranks with
    device-scope loads).  At least one step takes that path here; ranks per cluster and
    step equal the oracle's and the apply, which reads every reflector, T factor and W
    block these launches wrote, equals the oracle's within 1e-10.  A refactorization
    estimates the interfaces' steps from the previous ranks, which may move a step to or
    from that path; the factors come out the same bits either way."""
    p = gridgen.laplacian(shape)
    b = gridgen.rhs(np.random.default_rng(17), p.n, 3)
    an, fac = oracle_run(p, levels, 1e-2)
    s = gpu_factor(p, levels, 1e-2)
    st = s.stats()
    assert st["cpqr_one_launch_steps"] > 0, st
    assert rank_mismatches(s, an, fac) == 0
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    assert (st["s_top"], st["m_F"]) == (fac.stats["s_top"], fac.stats["m_F"])
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    assert np.array_equal(gpu_apply(s, b), z)
    s.close()


def test_refactor_same_handle():
    """A handle is refactored with new values and a new tolerance."""
    import torch as T
    p = gridgen.laplacian((10, 9, 8))
    b = gridgen.rhs(np.random.default_rng(1), p.n, 1)
    s = gpu_factor(p, 5, 1e-1)
    _, it1, _, _ = gpu_solve(s, b)
    s.factor(T.from_numpy(3.0 * p.values).to("cuda:0"), 1e-4)
    x, it2, rr, _ = gpu_solve(s, 3.0 * b)
    assert it2[0] <= it1[0] and rr[0] <= 1e-12


# ------------------------------------------------------------------ error paths
def test_not_spd_reported():
    from paper_1901_02971_amd import SpandError
    p = gridgen.laplacian((8, 8))
    vals = p.values.copy()
    vals[np.nonzero(p.colind == 0)[0][0]] = -4.0
    from paper_1901_02971_amd import Solver
    s = Solver.from_problem(p, 3)
    with pytest.raises(SpandError) as e:
        s.factor(torch.from_numpy(vals).to("cuda:0"), 1e-2)
    assert e.value.name == "SPAND_E_NOT_SPD"
    st = s.stats()
    assert st["fail_step"] == 1 and st["fail_phase"] == 0
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 3)
    with pytest.raises(O.NotSPD) as eo:
        O.factor(an, vals, 1e-2)
    assert (eo.value.step, eo.value.cluster) == (st["fail_step"], st["fail_cluster"])


def test_nonfinite_values_and_rhs():
    from paper_1901_02971_amd import Solver, SpandError
    p = gridgen.laplacian((8, 8))
    s = Solver.from_problem(p, 3)
    vals = p.values.copy()
    vals[5] = np.nan
    with pytest.raises(SpandError) as e:
        s.factor(torch.from_numpy(vals).to("cuda:0"), 1e-2)
    assert e.value.name == "SPAND_E_INVALID"
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    b = np.ones((p.n, 1))
    b[3] = np.inf
    with pytest.raises(SpandError) as e:
        gpu_solve(s, b)
    assert e.value.name == "SPAND_E_INVALID"


def test_noconv_reports_iterations():
    p = gridgen.laplacian((12, 12, 12))
    b = gridgen.rhs(np.random.default_rng(2), p.n, 2)
    s = gpu_factor(p, 6, 0.5)
    x, it, rr, st = gpu_solve(s, b, maxit=1, check=False)
    assert st == 3   # SPAND_E_NOCONV
    assert np.all(it == 1) and np.all(rr > 1e-12) and np.all(np.isfinite(x))


def test_pcg_breakdown_reported():
    """A residual norm that overflows is a breakdown, reported as such by both sides.
    b is the smoothest grid mode with ||b||^2 just below the FP64 maximum, so
    r.z = b^T M M^T b ~ ||b||^2 / lambda_min overflows in the first iteration."""
    from paper_1901_02971_amd import SpandError  # noqa: F401
    shape = (12, 12, 12)
    p = gridgen.laplacian(shape)
    i, j, k = (np.arange(s) + 1.0 for s in shape)
    mode = np.einsum("k,j,i->kji", np.sin(np.pi * k / 13), np.sin(np.pi * j / 13), np.sin(np.pi * i / 13)).ravel()
    b = (1.3e154 * mode / np.linalg.norm(mode))[:, None]
    assert np.isfinite(float(b[:, 0] @ b[:, 0]))
    an, fac = oracle_run(p, 6, 1e-2)
    with pytest.raises(O.Breakdown):
        O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    s = gpu_factor(p, 6, 1e-2)
    x, it, rr, st = gpu_solve(s, b, check=False)
    assert st == 7, st   # SPAND_E_BREAKDOWN
    assert it[0] == 1
    # the handle stays usable
    b2 = gridgen.rhs(np.random.default_rng(4), p.n, 1)
    _, it2, rr2, st2 = gpu_solve(s, b2)
    assert st2 == 0 and rr2[0] <= 1e-12


@pytest.mark.parametrize("fuse", [0, -1], ids=["fused128", "tiled"])
def test_apply_paths_match_oracle(fuse):
    """Interfaces of 65..128 dofs through the fused one-wave apply kernel (forced on
    with fuse128_min = 0) or through the tiled kernels (fuse128_min = -1): the apply
    equals the oracle's element by element, and the path counters show which ran."""
    p = gridgen.laplacian((24, 24, 24))
    b = gridgen.rhs(np.random.default_rng(12), p.n, 5)
    an, fac = oracle_run(p, 5, 1e-2)
    from paper_1901_02971_amd import Solver
    s = Solver.from_problem(p, 5)
    s.set_tuning(fuse128_min=fuse)
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    assert rank_mismatches(s, an, fac) == 0
    ai = s.stats()["apply_interfaces"]
    note(f"apply interfaces (fused <= 64, fused 65..128, tiled): {ai}")
    if fuse == 0:
        assert ai[1] > 0
    else:
        assert ai[1] == 0 and ai[2] > 0
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    x, it, rr, _ = gpu_solve(s, b)
    assert np.all(rr <= 1e-12)


@pytest.mark.parametrize("group", [1, 2, 4])
def test_cholesky_group_tuning_keeps_parity(group):
    """The trailing-update grouping of the blocked Cholesky (a tuning parameter)
    changes only the order of roundings: ranks stay the oracle's and the apply stays
    within 1e-10 of it."""
    p = gridgen.variable_coefficient((22, 20, 24), np.random.default_rng(41), -3, 3)
    b = gridgen.rhs(np.random.default_rng(42), p.n, 2)
    an, fac = oracle_run(p, 6, 1e-2)
    from paper_1901_02971_amd import Solver
    s = Solver.from_problem(p, 6)
    s.set_tuning(chol_group=group)
    assert s.tuning()["chol_group"] == group
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    assert rank_mismatches(s, an, fac) == 0
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()


@pytest.mark.parametrize("big_min,shape,levels", [(1, (24, 24, 24), 5), (60, (26, 23, 21), 6)],
                         ids=["all_big", "mixed"])
def test_large_interface_cpqr_matches_oracle(big_min, shape, levels):
    """The global-memory CPQR kernel (one cooperative launch per interface, the path
    of interfaces beyond the register layouts) forced on every interface of at
    least big_min dofs: ranks identical to the oracle's, the apply within 1e-10."""
    p = gridgen.variable_coefficient(shape, np.random.default_rng(61), -2, 2)
    b = gridgen.rhs(np.random.default_rng(62), p.n, 3)
    an, fac = oracle_run(p, levels, 1e-2)
    from paper_1901_02971_amd import Solver
    s = Solver.from_problem(p, levels)
    s.set_tuning(cpqr_big_min=big_min)
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    st = s.stats()
    note(f"big CPQR interfaces {st['cpqr_big_interfaces']}, register layouts {st['cpqr_interfaces']}")
    assert st["cpqr_big_interfaces"] > 0
    if big_min == 1:
        assert sum(st["cpqr_interfaces"]) == 0
    else:
        assert sum(st["cpqr_interfaces"]) > 0
    assert rank_mismatches(s, an, fac) == 0
    assert st["s_top"] == fac.stats["s_top"] and st["m_F"] == fac.stats["m_F"]
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    x, it, rr, _ = gpu_solve(s, b)
    _, it_ref, _ = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    assert np.all(np.abs(it - it_ref) <= 1) and np.all(rr <= 1e-12)


def test_gemm_tile_variants_agree_bit_for_bit():
    """Every output tile of the FP64 GEMM adds an entry's products in one order: the
    factorization, and so the apply, is the same bits whichever tile each GEMM class
    uses (the autotuner only reorders work)."""
    p = gridgen.variable_coefficient((22, 21, 20), np.random.default_rng(71), -2, 2)
    b = gridgen.rhs(np.random.default_rng(72), p.n, 2)
    from paper_1901_02971_amd import Solver
    vals = torch.from_numpy(p.values).to("cuda:0")
    zs = []
    for v in (0, 1, 2):
        s = Solver.from_problem(p, 6)
        s.set_tuning(gemm_syrk=v, gemm_chol=v, gemm_scale=v)
        s.factor(vals, 1e-2)
        zs.append(gpu_apply(s, b))
        s.close()
    assert np.array_equal(zs[0], zs[1]) and np.array_equal(zs[0], zs[2])


def test_autotune_and_cache(tmp_path, monkeypatch):
    """spand_autotune picks a tuning, leaves the handle factored with it (parity with
    the oracle unchanged), and stores the choice in SPAND_TUNE_CACHE, from which a
    second handle takes it without measuring."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SPAND_TUNE_CACHE", str(cache))
    p = gridgen.variable_coefficient((20, 19, 18), np.random.default_rng(73), -2, 2)
    b = gridgen.rhs(np.random.default_rng(74), p.n, 2)
    an, fac = oracle_run(p, 6, 1e-2)
    from paper_1901_02971_amd import Solver
    vals = torch.from_numpy(p.values).to("cuda:0")
    s = Solver.from_problem(p, 6)
    t1 = s.autotune(vals, 1e-2, nrhs=2, reps=1)
    note(f"autotune chose {t1}")
    assert s.tuning() == t1
    assert rank_mismatches(s, an, fac) == 0
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and " | " in lines[0]
    s2 = Solver.from_problem(p, 6)
    t2 = s2.autotune(vals, 1e-2, nrhs=2, reps=1)
    assert t2 == t1 and len(cache.read_text().splitlines()) == 1
    assert np.array_equal(gpu_apply(s2, b), z)


GRAPH = [
    ("permuted_grid_16x14x12", lambda: gridgen.permuted(gridgen.laplacian((16, 14, 12)), np.random.default_rng(7)), 6),
    ("knn_graph_2500", lambda: gridgen.knn_graph_laplacian(2500, 6, np.random.default_rng(8)), 6),
    ("var3d_16x15x14", lambda: gridgen.variable_coefficient((16, 15, 14), np.random.default_rng(9), -3, 3), 6),
]


@pytest.mark.parametrize("name,make,levels", GRAPH, ids=[c[0] for c in GRAPH])
def test_graph_separator_parity(name, make, levels):
    """Matrices analyzed from the graph alone (no coordinates): ranks identical to the
    oracle's, the apply within 1e-10 of it, iterations within +-1, relres <= 1e-12."""
    p = make()
    b = gridgen.rhs(np.random.default_rng(50), p.n, 3)
    an, fac = oracle_run(p, levels, 1e-2, geometry=False)
    s = gpu_factor(p, levels, 1e-2, geometry=False)
    assert rank_mismatches(s, an, fac) == 0
    assert s.stats()["s_top"] == fac.stats["s_top"] and s.stats()["m_F"] == fac.stats["m_F"]
    z = gpu_apply(s, b)
    zr = O.apply(fac, b)
    assert np.abs(z - zr).max() <= 1e-10 * np.abs(zr).max()
    x, it, rr, _ = gpu_solve(s, b)
    _, it_ref, _ = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    note(f"{name}: iters {it} oracle {it_ref}")
    assert np.all(np.abs(it - it_ref) <= 1) and np.all(rr <= 1e-12)


# ------------------------------------------------------------------ Schur-product precisions
@pytest.mark.parametrize("prec,bound", [(1, 1e-5), (2, 1e-4)], ids=["fp32", "bf16x3"])
def test_exact_factorization_reduced_precision(prec, bound):
    """With eps = 0 the FP32-MFMA and BF16x3 Schur products give an approximate
    inverse accurate to their precision; FP64 PCG still reaches 1e-12."""
    p = gridgen.laplacian((10, 9, 8))
    b = gridgen.rhs(np.random.default_rng(6), p.n, 2)
    s = gpu_factor(p, 5, 0.0, 0, prec)
    z = gpu_apply(s, b)
    x_ref = sla.cho_solve(sla.cho_factor(p.scipy().toarray()), b)
    err = np.abs(z - x_ref).max() / np.abs(x_ref).max()
    note(f"prec {prec}: exact-factorization apply error {err:.2e}")
    assert 1e-14 < err <= bound
    x, it, rr, _ = gpu_solve(s, b)
    assert np.all(it <= 3) and np.all(rr <= 1e-12)


@pytest.mark.parametrize("prec", [1, 2], ids=["fp32", "bf16x3"])
def test_c2_reduced_precision_iterations(prec):
    """32^3 Laplacian, eps = 1e-2: PCG iteration counts within +-1 of the FP64 oracle."""
    p, b, L = gridgen.config_problem("c2")
    an, fac = oracle_run(p, L, 1e-2)
    _, it_ref, _ = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    s = gpu_factor(p, L, 1e-2, 0, prec)
    x, it, rr, _ = gpu_solve(s, b)
    note(f"c2 prec {prec}: iters {it} oracle {it_ref} relres {rr}")
    assert np.all(np.abs(it - it_ref) <= 1) and np.all(rr <= 1e-12)


@pytest.mark.parametrize("make,levels,nrhs", [(lambda: gridgen.config_problem("c2")[0], 9, 1),
                                              (lambda: gridgen.variable_coefficient((14, 12, 10),
                                                                                    np.random.default_rng(31),
                                                                                    -3, 3), 5, 3)])
def test_apply_graph_matches_eager(make, levels, nrhs):
    """PCG with the apply replayed from a captured graph (eager SpMV, dots, updates and
    host synchronisations between the replays) gives bit-identical iterates to
    launching the apply kernel by kernel, also on a second solve (a new capture)."""
    p = make()
    b = gridgen.rhs(np.random.default_rng(32), p.n, nrhs)
    s = gpu_factor(p, levels, 1e-2)
    x_g, it_g, rr_g, _ = gpu_solve(s, b)
    assert s.stats()["apply_graph"] == 1
    x_g2, it_g2, _, _ = gpu_solve(s, b)
    s.set_apply_graph(False)
    x_e, it_e, rr_e, _ = gpu_solve(s, b)
    assert s.stats()["apply_graph"] == 0
    assert np.array_equal(it_g, it_e) and np.array_equal(it_g2, it_e)
    assert np.array_equal(x_g, x_e) and np.array_equal(x_g2, x_e)
    assert np.array_equal(rr_g, rr_e) and rr_e.max() <= 1e-12
