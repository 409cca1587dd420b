"""GPU: the no-allocation entry point ez_lattice_sums_noalloc (through the C ABI)
against ez_lattice_sums on the same inputs: two calls in a row, the second with
a smaller input (the static scratch keeps the first call's contents), and a
request beyond the scratch's size refused on the host."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ATM_NU = [-1.0, 1.0, 3.0, 5.0]
ATM_TERMS = [(0, 1.0 / 24.0, [(2, 3)]), (0, -3.0 / 16.0, [(0, 1), (3, 2)]), (0, 3.0 / 8.0, [(1, 1), (2, 1), (3, 1)])]


@pytest.fixture(scope="module")
def ez():
    import paper_2504_11989_amd as ez
    ez.version()
    return ez


def both(ez, A, nu, terms, n_res, specs):
    ref, st_ref = ez.lattice_sums(A, nu, terms, n_res, specs, with_status=True)
    got, st = ez.lattice_sums(A, nu, terms, n_res, specs, with_status=True, noalloc=True)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy(), st.cpu().numpy(), st_ref.cpu().numpy()


def test_noalloc_matches_lattice_sums_two_calls(ez):
    from paper_2504_11989_amd.batch import SCAN_NU, SCAN_TERMS
    # 1: the three-lattice ATM workload on the full plan (half-term tail workgroups included)
    lat = np.stack([W.sc(), W.fcc(), W.bcc()])
    got, ref, st, st_ref = both(ez, lat, ATM_NU, ATM_TERMS, 1, W.SPEC_FULL_3D)
    assert np.array_equal(st, np.zeros(3, np.int32)) and np.array_equal(st_ref, st)
    assert np.array_equal(got, ref), (got, ref)
    # 2: a smaller call right after: two bct lattices, uneven small plans, scan program
    ca, nside, A = W.c3_scan()
    specs = [W.c3_spec(16, lam=1.3), W.c3_spec(20, lam=1.3)]
    got, ref, st, _ = both(ez, A[:2], SCAN_NU, SCAN_TERMS, 5, specs)
    assert np.array_equal(st, np.zeros(2, np.int32))
    assert np.array_equal(got, ref), (got, ref)
    # 3: the first call again (its plan is uploaded again)
    got, ref, _, _ = both(ez, lat, ATM_NU, ATM_TERMS, 1, W.SPEC_FULL_3D)
    assert np.array_equal(got, ref)


def test_noalloc_rejects_beyond_scratch(ez):
    ca, nside, A = W.c3_scan()
    with pytest.raises(ez.EzError, match="no-allocation scratch"):
        ez.lattice_sums(A[:512], ATM_NU, ATM_TERMS, 1, W.SPEC_FULL_3D, noalloc=True)
