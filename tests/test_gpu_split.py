"""GPU tests of the CPU/GPU split of host-resident packets
(hydro_stream_set_cpu_share): the last packets of a stream are advanced by
host threads with the host FP64 kernel while the GPU streams the others.

FP64: any share gives the same arena, bit for bit, as the GPU-only stream
and the device batch (the host kernel runs the FP64 GPU path's operations
in its order), and the oracle's to 1e-12.  Mixed GPU packets with FP64 host
packets: within the mixed bar of the oracle.  A non-physical state in a host
packet follows the failure contract.  A method variant takes no share."""
import numpy as np
import pytest

from gpu_util import l1_rho, rel_err, to_dev, to_host
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


@pytest.fixture(scope="module")
def uneven():
    P = I.uneven(nblocks=150, nsteps=8)
    R = P.U0.copy()
    _, t = O.run(P.mesh, R, P.nsteps, P.cfl, P.gamma)
    return P, R, t


def _stream(P, prec, cpu_packets, nthreads=4, nslots=2, U0=None, unit=0):
    import torch

    host = torch.from_numpy((P.U0 if U0 is None else U0).copy()).pin_memory()
    hs = H.HostStream(P.mesh, host, P.packets, prec, nslots)
    if unit:
        hs.set_unit_bytes(unit)
    if cpu_packets:
        hs.set_cpu_share(cpu_packets, nthreads)
    return host, hs


def test_split_fp64_bitwise_and_oracle(uneven):
    P, R, t_ref = uneven
    outs = []
    # the last case: GPU packets merged into transfer units of >= 1 MiB
    for k, unit in ((0, 0), (5, 0), (len(P.packets) // 2, 0), (len(P.packets), 0), (5, 1 << 20)):
        host, hs = _stream(P, H.FP64, k, unit=unit)
        t = hs.run(P.nsteps, P.cfl, P.gamma)
        hs.close()
        outs.append((host.numpy().copy(), t))
    for U, t in outs:
        assert np.array_equal(U, outs[0][0]) and t == outs[0][1]
    assert rel_err(P.mesh, outs[0][0], R) <= 1e-12
    assert abs(outs[0][1] - t_ref) <= 1e-12 * t_ref


def test_split_mixed_within_bar(uneven):
    P, R, t_ref = uneven
    host, hs = _stream(P, H.FP32_FP64, len(P.packets) // 3)
    t = hs.run(P.nsteps, P.cfl, P.gamma)
    hs.close()
    assert l1_rho(P.mesh, host.numpy(), R) <= 1e-5
    assert abs(t - t_ref) <= 1e-6 * t_ref


def test_split_failure_contract(uneven):
    """A non-physical cell in a host packet: ENONPHYS naming its block, and
    the host arena keeps the initial state (nothing advanced)."""
    P = uneven[0]
    U0 = P.U0.copy()
    bad = int(P.packets[-1][0])
    P.mesh.block_view(U0, bad)[4, 0, 1, 2] = 0.0
    host, hs = _stream(P, H.FP64, 2, U0=U0)
    with pytest.raises(H.HydroError) as e:
        hs.run(3, P.cfl, P.gamma)
    hs.close()
    assert e.value.code == H.ENONPHYS and f"block {bad}" in str(e.value)
    assert np.array_equal(host.numpy(), U0)


def test_split_refuses_variants(uneven):
    P = uneven[0]
    host, hs = _stream(P, H.FP64 | H.EINFELDT, 0)
    with pytest.raises(H.HydroError) as e:
        hs.set_cpu_share(2, 2)
    assert e.value.code == H.EINVAL
    with pytest.raises(H.HydroError):
        _stream(P, H.FP64, len(P.packets) + 1)
    hs.close()
