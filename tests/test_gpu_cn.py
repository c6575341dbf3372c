"""Crank-Nicolson on the GPU (chebtd_crank_nicolson, eq. (CN)) against the
oracle's sequential Thomas solve on the same seeded inputs."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import assert_state_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def cheb():
    import paper_0907_3022_amd as P
    P.load_library()
    return P


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(torch, cheb, V, dx, psi0, dt, S):
    ctx = cheb.Context()
    ctx.chain1d(torch.from_numpy(V).cuda(), dx)
    psi = torch.from_numpy(psi0.copy()).cuda()
    ctx.crank_nicolson(psi, dt, S)
    torch.cuda.synchronize()
    return psi.cpu().numpy()


# ragged chain lengths: fewer sites than threads, one per thread, one past
# that (two per thread), partly filled chunks, the 4096 maximum
@pytest.mark.parametrize("n", [2, 37, 64, 256, 257, 1000, 2048, 4095, 4096])
@pytest.mark.parametrize("S", [1, 7])
@pytest.mark.parametrize("state", ["packet", "dense"])
def test_cn_matches_oracle(torch, cheb, n, S, state):
    x, dx, V, psi0 = W.double_well_inputs(n)
    if state == "dense":  # every site of every thread's chunk carries amplitude
        psi0 = W.random_state(n, 300 + n)
    dt = 0.05
    ref = O.crank_nicolson_1d(V, dx, psi0, dt, S)
    got = run(torch, cheb, V, dx, psi0, dt, S)
    assert_state_close(got, ref)


def test_cn_double_well_workload(torch, cheb):
    # the Sect. 3.1 double well at its full 4096-point grid, with the
    # Chebyshev step dt = 0.5 split into 50 CN steps
    p = W.DOUBLE_WELL.params
    x, dx, V, psi0 = W.double_well_inputs(p["n"], p["xmin"], p["xmax"], p["a"], p["b"],
                                          p["x0"], p["sigma"], p["k0"])
    ref = O.crank_nicolson_1d(V, dx, psi0, 0.01, 50)
    got = run(torch, cheb, V, dx, psi0, 0.01, 50)
    assert rel_l2(got, ref) <= 1e-10
    # CN is unitary: the norm stays 1 to rounding
    assert abs(np.linalg.norm(got) - 1.0) <= 1e-12


def test_cn_zero_steps_and_errors(torch, cheb):
    x, dx, V, psi0 = W.double_well_inputs(100)
    got = run(torch, cheb, V, dx, psi0, 0.1, 0)
    np.testing.assert_array_equal(got, psi0)
    ctx = cheb.Context()
    ctx.chain1d(torch.from_numpy(V).cuda(), dx)
    psi = torch.from_numpy(psi0.copy()).cuda()
    with pytest.raises(cheb.ChebError):
        ctx.crank_nicolson(psi, -0.1, 3)
    # a chain longer than one workgroup holds in registers is refused
    xb, dxb, Vb, pb = W.double_well_inputs(1 << 14)
    big = cheb.Context()
    big.chain1d(torch.from_numpy(Vb).cuda(), dxb)
    with pytest.raises(cheb.ChebError, match="n <= 4096"):
        big.crank_nicolson(torch.from_numpy(pb).cuda(), 0.1, 1)
    # only the chain has a CN path
    eps, pr = W.ribbon_inputs(8, 40, 0.5, 3)
    rib = cheb.Context()
    rib.honeycomb(8, 40, torch.from_numpy(eps).cuda())
    with pytest.raises(cheb.ChebError):
        rib.crank_nicolson(torch.from_numpy(pr).cuda(), 0.1, 1)
