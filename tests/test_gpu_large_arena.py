"""GPU parity on an arena past 2^31 elements.

105000 self-periodic blocks of 16^3 (2.15e9 doubles, 17.2 GB, plus as much
first-stage scratch): every block starts at one uniform state except three
blocks with a seeded smooth random state, the first, the middle and the last
block of the arena; the last starts beyond element 2^31.  After two batched
steps (graph path, 103 packets) in each precision:
  * the three blocks and one uniform block match the oracle run on a mesh of
    the same four blocks (its time steps are the same: the largest CFL rate
    over all blocks is the largest over these four), FP64 <= 1e-12 relative
    per cell (floored as in the other parity tests) and in the simulated
    time, mixed FP32/FP64 L1(rho) <= 1e-5;
  * every other block still holds the uniform state bit for bit (a uniform
    state is a steady state of the scheme, exactly, in both precisions).
"""
import numpy as np
import pytest

from gpu_util import l1_rho, rel_err
from oracle import oracle as O
from paper_2507_09337_amd import hydro as H
from paper_2507_09337_amd import inputs as I

pytestmark = pytest.mark.gpu

GAMMA = 1.4
CFL = 0.4
NSTEPS = 2
NB = 105000
CELLS = 16 ** 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def test_arena_past_2_31_elements():
    import torch

    mesh = I.independent_blocks([16] * NB)
    sample = [0, NB // 2, NB - 1]
    assert int(mesh.offset[NB - 1]) > 2 ** 31 and mesh.arena_len > 2 ** 31
    # the oracle's mesh: block 0 uniform, blocks 1..3 the perturbed ones
    small = I.independent_blocks([16] * 4)
    U_small = I.random_smooth_state(small, seed=11, gamma=GAMMA)
    uni = I.uniform_state(I.independent_blocks([16]), gamma=GAMMA)
    U_small[: uni.size] = uni
    R = U_small.copy()
    _, t_ref = O.run(small, R, NSTEPS, CFL, GAMMA)

    arena = torch.empty(mesh.arena_len, dtype=torch.float64, device="cuda")
    blocks = arena.view(NB, 5, CELLS)
    u = torch.from_numpy(uni.reshape(5, CELLS)).cuda()
    per = U_small.reshape(4, 5, CELLS)
    others = torch.ones(NB, dtype=torch.bool, device="cuda")
    others[sample] = False
    for prec in (H.FP64, H.FP32_FP64):
        blocks.copy_(u.expand(NB, 5, CELLS))
        for k, b in enumerate(sample):
            blocks[b].copy_(torch.from_numpy(per[k + 1]).cuda())
        m = H.Mesh(mesh, arena)
        bt = H.Batch([H.Packet(m, ids, prec) for ids in I.contiguous_packets(NB, 1024)])
        t = bt.run(NSTEPS, CFL, GAMMA)
        torch.cuda.synchronize()
        # one uniform block (the one just before the last) in place of the oracle mesh's block 0
        G = np.concatenate([blocks[b].cpu().numpy().ravel() for b in [NB - 2] + sample])
        changed = int((blocks != u).any(dim=2).any(dim=1)[others].sum().item())
        bt.close()
        m.close()
        assert changed == 0, (prec, changed)
        if prec == H.FP64:
            assert abs(t - t_ref) <= 1e-12 * t_ref, (t, t_ref)
            assert rel_err(small, G, R) <= 1e-12
        else:
            assert l1_rho(small, G, R) <= 1e-5
