"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments without touching a GPU, and its host
Holstein builder agrees exactly with the oracle's independent builder."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_0907_3022_amd import _lib as L
    try:
        return L, L.lib()
    except L.ChebError as e:  # not built
        pytest.fail(str(e))


def header_functions():
    src = open(os.path.join(ROOT, "include", "chebtd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chebtd_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    names = header_functions()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    # the binding knows every declared entry point and nothing else
    assert sorted(L.exported_names()) == names


def test_version():
    _, lib = _lib()
    assert lib.chebtd_version() >= 10000


def test_null_context_is_rejected_without_gpu():
    L, lib = _lib()
    dummy = C.c_void_p(0)
    assert lib.chebtd_h_chain1d(None, 10, 0.1, dummy) == L.E_ARG
    assert lib.chebtd_set_bounds(None, 0.0, 1.0, 0.01) == L.E_ARG
    assert lib.chebtd_propagate(None, dummy, 1, None, None, 0) == L.E_ARG
    assert lib.chebtd_adjoint(None, dummy, dummy) == L.E_ARG
    assert lib.chebtd_adjoint_run(None, 1, dummy, dummy) == L.E_ARG
    rid = C.c_int64(7)
    assert lib.chebtd_checkpoint_run(None, C.byref(rid)) == L.E_ARG
    assert lib.chebtd_batch_propagate(None, None, 1, 0) == L.E_ARG
    assert lib.chebtd_create(None, None) == L.E_ARG
    assert "null" in L.last_error(None)
    assert lib.chebtd_destroy(None) == L.OK
    assert lib.chebtd_dim(None) == 0


@pytest.mark.parametrize("L_sites,nph,periodic", [(3, 2, True), (4, 3, False), (5, 3, True),
                                                 (1, 6, False), (10, 3, True)])
def test_host_holstein_builder_matches_oracle(L_sites, nph, periodic):
    from paper_0907_3022_amd import holstein_csr_host, holstein_occupations
    rng = np.random.default_rng(L_sites * 7 + nph)
    g = rng.uniform(0.2, 1.5, L_sites)
    Delta = rng.uniform(-1.0, 1.0, L_sites)
    rowptr, col, val = holstein_csr_host(L_sites, nph, 1.0, 1.3, g, Delta, periodic)
    orow, ocol, oval = O.holstein(L_sites, nph, 1.0, 1.3, g, Delta, periodic).csr()
    np.testing.assert_array_equal(rowptr, orow)
    np.testing.assert_array_equal(col.astype(np.int64), ocol)
    # identical expressions on both sides: exact agreement
    np.testing.assert_array_equal(val, oval)
    np.testing.assert_array_equal(holstein_occupations(L_sites, nph),
                                  O.holstein_occupations(L_sites, nph))


@pytest.mark.parametrize("L_sites,nph", [(10, 6), (7, 9), (1, 40)])
def test_host_holstein_tables_match_oracle_order(L_sites, nph):
    # large enough that the library splits the basis over host threads and
    # starts each thread by unranking
    from paper_0907_3022_amd import holstein_occupations
    np.testing.assert_array_equal(holstein_occupations(L_sites, nph),
                                  O.holstein_occupations(L_sites, nph))


def test_paper_scale_polaron_dimension(golden_dir):
    # Sect. 3.3: 18 sites, at most 11 phonons -> D = 6.2e8
    import ctypes as C
    import json
    L, lib = _lib()
    g = json.load(open(os.path.join(golden_dir, "paper_values.json")))["polaron"]
    cnt = C.c_int64()
    assert lib.chebtd_holstein_occupations(g["L"], g["nph"], C.byref(cnt), None) == L.OK
    assert cnt.value * g["L"] == 622_751_220
    assert float(f"{cnt.value * g['L']:.2g}") == g["D_tot"]


def test_host_holstein_config3_dimension_and_nnz():
    from paper_0907_3022_amd import holstein_csr_host
    rowptr, col, val = holstein_csr_host(10, 10, 1.0, 1.0, np.sqrt(0.5), 0.0, True)
    n = rowptr.size - 1
    assert n == 1_847_560
    nnz = rowptr[-1]
    # diagonal + two hops per row, plus one creation where the total is below
    # N_ph and one annihilation per occupied site: exactly 4 per row on average
    assert nnz == 4 * n
    assert np.all(np.diff(rowptr) >= 3) and np.all(np.diff(rowptr) <= 5)


def test_host_holstein_rejects_bad_arguments():
    from paper_0907_3022_amd import ChebError, holstein_csr_host
    with pytest.raises(ChebError):
        holstein_csr_host(2, 3, 1.0, 1.0, 0.5, 0.0, True)  # ring needs L >= 3
    with pytest.raises(ChebError):
        holstein_csr_host(0, 3, 1.0, 1.0, 0.5, 0.0, False)
