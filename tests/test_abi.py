"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
its host-only analysis (Algorithm 2 + symbolic factorization) equals the oracle's
bit for bit.  No compute call touches a GPU here."""
import ctypes

import numpy as np
import pytest

import gridgen
from oracle import spand_oracle as O
from paper_1901_02971_amd import spand as S

DECLARED = ["spand_analyze", "spand_factor", "spand_solve", "spand_apply", "spand_set_stream",
            "spand_set_apply_graph", "spand_get_stats", "spand_set_tuning", "spand_get_tuning", "spand_autotune",
            "spand_set_variant", "spand_get_variant",
            "spand_apply_noalloc", "spand_get_permutation",
            "spand_get_ordering", "spand_step_counts", "spand_step_structure", "spand_step_ranks",
            "spand_factor_batch", "spand_solve_batch", "spand_error_string", "spand_destroy"]


def test_header_declares_expected_symbols():
    assert S.exported_symbols() == sorted(DECLARED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(S.library_path())
    for name in S.exported_symbols():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("cname,mirror", [("spand_stats", "Stats"), ("spand_tuning", "Tuning")])
def test_stats_struct_matches_header(tmp_path, cname, mirror):
    """The ctypes mirrors of the header's structs have the size and field offsets the
    C compiler gives them (a C program built with the host compiler prints them)."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    M = getattr(S, mirror)
    fields = [name for name, _ in M._fields_]
    src = ["#include <stddef.h>", "#include <stdio.h>", '#include "spand.h"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({cname}));']
    src += [f'  printf("%zu\\n", offsetof({cname}, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "stats.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "stats"
    r = subprocess.run([cc, "-std=c11", "-I", inc, str(c), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(M)
    for f, off in zip(fields, vals[1:]):
        assert getattr(M, f).offset == off, f


def _graph_problems():
    return [("grid2d", gridgen.laplacian((33, 20)), 6),
            ("grid3d", gridgen.laplacian((12, 10, 9)), 6),
            ("permuted3d", gridgen.permuted(gridgen.laplacian((10, 11, 12)), np.random.default_rng(5)), 6),
            ("knn", gridgen.knn_graph_laplacian(2000, 7, np.random.default_rng(6)), 7)]


@pytest.mark.parametrize("name,p,levels", _graph_problems(), ids=[c[0] for c in _graph_problems()])
def test_graph_separator_analyze_bit_exact_vs_oracle(name, p, levels):
    """Without coordinates (dim = 0) the library's level-structure separator, cluster
    keys, block patterns and colouring equal the oracle's bit for bit."""
    lib = S.Solver.from_problem(p, levels, geometry=False)
    an = O.Analysis(p.n, p.rowptr, p.colind, None, levels)
    Sg, Lg, Rg = lib.ordering()
    assert np.array_equal(Sg, an.S) and np.array_equal(Lg, an.L) and np.array_equal(Rg, an.R)
    for t, st in enumerate(an.steps, start=1):
        g = lib.step_structure(t)
        assert np.array_equal(g["keys"], st.keys)
        assert np.array_equal(g["colour"], st.colour)
        assert [tuple(x) for x in g["after"]] == [tuple(x) for x in st.after]


@pytest.mark.parametrize("shape,levels,geometry", [((7, 7), 3, True), ((12, 10, 9), 6, True),
                                                   ((16, 16), 5, False), ((10, 11, 12), 6, False)])
def test_permutation_bit_exact_vs_oracle(shape, levels, geometry):
    """The nested-dissection elimination order equals the oracle's, is a permutation,
    and eliminates every separator after the separators below it."""
    p = gridgen.laplacian(shape)
    lib = S.Solver.from_problem(p, levels, geometry)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords if geometry else None, levels)
    perm = lib.permutation()
    assert np.array_equal(perm, O.nd_permutation(an))
    assert np.array_equal(np.sort(perm), np.arange(p.n))
    lv = O.lev_of(an.S)[perm]
    assert np.all(np.diff(lv) <= 0)   # deeper levels first


def test_graph_separator_argument_checks():
    p = gridgen.laplacian((5, 5))
    with pytest.raises(S.SpandError):
        S.Solver(p.n, p.rowptr, p.colind, np.zeros((p.n, 0)), 3)   # dim 0 array is not NULL


CASES = [((7, 7), 3), ((6, 4), 2), ((16, 16), 5), ((64, 64), 6), ((9, 7, 6), 4), ((8, 8, 8), 5),
         ((24, 31, 40), 7), ((32, 32, 32), 9), ((5, 5, 5), 1), ((3, 2), 4)]


@pytest.mark.parametrize("shape,levels", CASES)
def test_analyze_bit_exact_vs_oracle(shape, levels):
    p = gridgen.laplacian(shape)
    lib = S.Solver.from_problem(p, levels)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels)
    Sg, Lg, Rg = lib.ordering()
    assert np.array_equal(Sg, an.S) and np.array_equal(Lg, an.L) and np.array_equal(Rg, an.R)
    for t, st in enumerate(an.steps, start=1):
        g = lib.step_structure(t)
        assert np.array_equal(g["keys"], st.keys)
        assert g["ne"] == st.n_elim and g["level"] == st.level
        assert np.array_equal(g["parent"], st.parent)
        if st.sparsify:
            assert np.array_equal(g["colour"], st.colour)
        assert np.array_equal(g["before"], np.array(st.blocks, dtype=np.int32).reshape(-1, 2))
        assert np.array_equal(g["after"], np.array(st.after, dtype=np.int32).reshape(-1, 2))


def test_analyze_bit_exact_variable_coefficient_config3_shape():
    """The 64^3 variable-coefficient workload at its real size and depth (10 levels)."""
    p = gridgen.variable_coefficient((64, 64, 64), np.random.default_rng(3), -3, 3)
    lib = S.Solver.from_problem(p, 10)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 10)
    Sg, Lg, Rg = lib.ordering()
    assert np.array_equal(Sg, an.S) and np.array_equal(Lg, an.L) and np.array_equal(Rg, an.R)
    for t, st in enumerate(an.steps, start=1):
        g = lib.step_structure(t)
        assert np.array_equal(g["keys"], st.keys) and np.array_equal(g["parent"], st.parent)
        assert np.array_equal(g["after"], np.array(st.after, dtype=np.int32).reshape(-1, 2))


def _expect(status_name, fn):
    with pytest.raises(S.SpandError) as e:
        fn()
    assert e.value.name == status_name


def test_analyze_rejects_bad_input():
    p = gridgen.laplacian((5, 5))
    _expect("SPAND_E_INVALID", lambda: S.Solver(p.n, p.rowptr, p.colind, p.coords, 0))
    bad = p.colind.copy()
    bad[1] = bad[0]    # not strictly increasing
    _expect("SPAND_E_INVALID", lambda: S.Solver(p.n, p.rowptr, bad, p.coords, 2))
    # non-symmetric pattern: drop the (0, 1) entry but keep (1, 0)
    rp = p.rowptr.copy()
    keep = np.ones(len(p.colind), bool)
    keep[1] = False
    rp[1:] -= 1
    _expect("SPAND_E_INVALID", lambda: S.Solver(p.n, rp, p.colind[keep], p.coords, 2))
    c = p.coords.copy()
    c[3, 0] = np.nan
    _expect("SPAND_E_INVALID", lambda: S.Solver(p.n, p.rowptr, p.colind, c, 2))
    _expect("SPAND_E_INVALID", lambda: S.Solver(p.n, p.rowptr, p.colind, np.zeros((p.n, 4)), 2))


def test_solve_before_factor_is_state_error():
    """No GPU work happens: the state check precedes every device call."""
    p = gridgen.laplacian((5, 5))
    lib = S.Solver.from_problem(p, 2)
    lib_c = S.load_library()
    it = np.zeros(1, np.int32)
    rr = np.zeros(1)
    st = lib_c.spand_solve(lib._h, 1, 8, 16, 1e-12, 10, it.ctypes.data, rr.ctypes.data)
    assert S.STATUS[st] == "SPAND_E_STATE"


def test_batch_rejects_bad_handle_lists():
    """Argument checks of the batched calls happen before any device work."""
    lib = S.load_library()
    p = gridgen.laplacian((6, 5))
    a = S.Solver.from_problem(p, 3)
    hs = (ctypes.c_void_p * 2)(a._h.value, a._h.value)
    vals = (ctypes.c_void_p * 2)(None, None)
    assert lib.spand_factor_batch(2, hs, vals, 1e-2, 0, 0) == 1  # repeated handle
    assert b"twice" in lib.spand_error_string(None)
    assert lib.spand_factor_batch(0, hs, vals, 1e-2, 0, 0) == 1
    nul = (ctypes.c_void_p * 1)(None)
    assert lib.spand_factor_batch(1, nul, vals, 1e-2, 0, 0) == 1
    it = np.zeros(2, np.int32)
    rr = np.zeros(2)
    assert lib.spand_solve_batch(2, hs, 1, vals, vals, 1e-12, 10, it.ctypes.data, rr.ctypes.data) == 1


def test_variant_selection_host_only():
    """spand_set_variant / spand_get_variant touch no GPU: the default is OrthS, the
    three variants round-trip, an unknown value is refused and leaves the choice."""
    p = gridgen.laplacian((6, 5))
    s = S.Solver.from_problem(p, 2)
    assert s.variant() == "OrthS"
    for v in ("In", "InS", "OrthS", "In"):
        s.set_variant(v)
        assert s.variant() == v
    lib = S.load_library()
    assert S.STATUS[lib.spand_set_variant(s._h, 3)] == "SPAND_E_INVALID"
    assert S.STATUS[lib.spand_set_variant(None, 0)] == "SPAND_E_INVALID"
    assert s.variant() == "In"
    s.close()
