"""The fixed-scratch D cotangent (dg_volume_grad_d_noalloc) against dg_volume_grad_d.

Two calls in a row per order, the second with a smaller problem, so the second
call runs over scratch that still holds the first call's partial sums; each
result must equal dg_volume_grad_d's bit for bit (same partition of the
columns, same kernels) and meet the FP64 criteria against the oracle.  An empty
problem writes zeros; a problem too large for the scratch is rejected.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1503_07659_amd import dgvol, synth
from parity import check_planes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _problem(N, K, F, seed):
    Np = oracle.num_nodes(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed))
    u = synth.fields(K, F, Np, seed + 1, "uniform")
    gout = synth.fields(K, 3 * F, Np, seed + 2, "normal").reshape(K, 3, F, Np).transpose(1, 0, 2, 3).copy()
    return G, u, gout


def _cond(G, u, gout):
    """sum over columns of |W_a| (x) |u|: the condition scale of every entry of gD."""
    return oracle.volume_grad_d(np.abs(G), np.abs(u), np.abs(gout))


# (order, first K, second K, F): the second problem is smaller; at orders 6 and 7 both fit the
# 64 MiB scratch (K*F <= 50 688 and <= 24 832)
CASES = [(1, 40000, 3001, 3), (3, 20000, 1777, 3), (4, 30000, 2500, 5), (5, 9000, 1200, 3),
         (6, 16000, 900, 3), (7, 8000, 601, 3)]


@pytest.mark.parametrize("N,K1,K2,F", CASES)
def test_noalloc_matches_workspace_entry(N, K1, K2, F):
    Np = oracle.num_nodes(N)
    for call, K in enumerate((K1, K2)):
        _say(f"grad_d_noalloc N={N} call={call} K={K} F={F}")
        G, u, gout = _problem(N, K, F, 6000 + 10 * N + call)
        Gd, ud, gd = dev(G), dev(u), dev(gout)
        ref_lib = dgvol.dg_volume_grad_d(Gd, ud, gd)
        got = torch.full((3, Np, Np), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_volume_grad_d_noalloc(Gd, ud, gd, got)
        torch.cuda.synchronize()
        got_h, ref_h = got.cpu().numpy(), ref_lib.cpu().numpy()
        assert np.array_equal(got_h, ref_h), f"call {call}: differs from dg_volume_grad_d"
        check_planes(got_h, oracle.volume_grad_d(G, u, gout), _cond(G, u, gout), what="gD")


def test_noalloc_empty_and_too_large():
    Np = 35
    gD = torch.full((3, Np, Np), float("nan"), dtype=torch.float64, device="cuda")
    e = torch.empty((0, 3, Np), dtype=torch.float64, device="cuda")
    dgvol.dg_volume_grad_d_noalloc(torch.empty((0, 9), dtype=torch.float64, device="cuda"), e,
                                   torch.empty((3, 0, 3, Np), dtype=torch.float64, device="cuda"), gD)
    torch.cuda.synchronize()
    assert (gD.cpu().numpy() == 0).all()
    # order 7 with one column more than the scratch holds: rejected before any launch
    K = 24833
    G = torch.zeros((K, 9), dtype=torch.float64, device="cuda")
    u = torch.zeros((K, 1, 120), dtype=torch.float64, device="cuda")
    g = torch.zeros((3, K, 1, 120), dtype=torch.float64, device="cuda")
    gD7 = torch.full((3, 120, 120), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(dgvol.DGVolError) as ei:
        dgvol.dg_volume_grad_d_noalloc(G, u, g, gD7)
    assert ei.value.status == dgvol.DG_ESCRATCH
    torch.cuda.synchronize()
    assert (gD7.cpu().numpy() == 7.0).all()
