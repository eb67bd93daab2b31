"""GPU: spand_apply_noalloc (the apply on the library's fixed device scratch, for
callers that cannot allocate) against spand_apply on the same handle, through the
C ABI: equal bit for bit on two calls in a row, the second with a smaller input
(a smaller grid and fewer right-hand sides), and a request beyond the fixed array
rejected with SPAND_E_INVALID before anything runs."""
import ctypes as C

import numpy as np
import pytest

import gridgen
from paper_1901_02971_amd import Solver, spand
from tests.gpu_util import note, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note(request.node.nodeid)


def _noalloc(lib, s, r, z):
    fn = lib.spand_apply_noalloc
    fn.restype = C.c_int32
    fn.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    nrhs = r.shape[0]
    return fn(s._h, nrhs, r.data_ptr(), z.data_ptr())


def test_apply_noalloc_matches_apply():
    lib = spand.load_library()
    cases = [(gridgen.variable_coefficient((20, 19, 18), np.random.default_rng(81), -2, 2), 6, 3),
             (gridgen.variable_coefficient((12, 11, 10), np.random.default_rng(82), -2, 2), 5, 1)]
    for p, levels, nrhs in cases:   # the second call has the smaller input
        s = Solver.from_problem(p, levels)
        s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
        r = to_dev(gridgen.rhs(np.random.default_rng(83), p.n, nrhs))
        z_ref = torch.empty_like(r)
        s.apply(r, z_ref)
        z = torch.full_like(r, np.nan)
        st = _noalloc(lib, s, r, z)
        assert st == 0, lib.spand_error_string(s._h)
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref), f"n={p.n} nrhs={nrhs}"
        note(f"n={p.n} nrhs={nrhs}: scratch {s.stats()['apply_scratch_per_rhs'] * nrhs} doubles")
        s.close()


def test_apply_noalloc_rejects_oversized_request():
    lib = spand.load_library()
    p = gridgen.variable_coefficient((12, 11, 10), np.random.default_rng(84), -2, 2)
    s = Solver.from_problem(p, 5)
    s.factor(torch.from_numpy(p.values).to("cuda:0"), 1e-2)
    per = s.stats()["apply_scratch_per_rhs"]
    nrhs = (8 << 20) // per + 1   # one right-hand side beyond the fixed array
    r = torch.zeros((nrhs, p.n), dtype=torch.float64, device="cuda:0")
    z = torch.zeros_like(r)
    st = _noalloc(lib, s, r, z)
    assert st == 1   # SPAND_E_INVALID
    assert b"needs" in lib.spand_error_string(s._h)
    assert torch.count_nonzero(z).item() == 0
    # the handle still works, through both entry points
    r1 = to_dev(gridgen.rhs(np.random.default_rng(85), p.n, 1))
    z1 = torch.empty_like(r1)
    s.apply(r1, z1)
    z2 = torch.empty_like(r1)
    assert _noalloc(lib, s, r1, z2) == 0
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    s.close()
