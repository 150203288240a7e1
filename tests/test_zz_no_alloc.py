"""The allocation-free operator application (ovs_apply_noalloc): the same
kernels as ovs_apply with the staging fields in the library's fixed
per-device scratch.  Its results must equal ovs_apply's bit for bit, on two
calls in a row (the second with a smaller input, so stale scratch contents
from the first would show), and a request beyond the scratch's size must be
rejected on the host."""
import numpy as np
import pytest

import synth
from oracle import dirac

from gpu_util import rel, say, to_dev

pytestmark = pytest.mark.gpu
MW = -1.5


def _lattice(dims, prec, seed, mu):
    import paper_0810_4228_amd as ovs
    lat = ovs.Lattice(dims, precision=prec)
    lat.set_links(to_dev(synth.random_links(dims, 0.5, seed=seed)))
    lat.set_params(MW, mu)
    return lat


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_equals_apply_two_calls(prec):
    import torch
    calls = [((4, 4, 6, 8), 5, "A"), ((4, 4, 4, 4), 2, "A_dag")]  # second: smaller
    for dims, nrhs, op in calls:
        lat = _lattice(dims, prec, 11, 0.35)
        x = to_dev(synth.gaussian_sources(dims, nrhs, seed=12))
        ref = lat.apply(op, x)
        out = torch.full_like(x, float("nan"))
        lat.apply_noalloc(op, x, out)
        torch.cuda.synchronize()
        same = bool(torch.equal(out, ref))
        U = synth.random_links(dims, 0.5, seed=11)
        A = dirac.csr_A(dims, U, MW, 0.35 if op == "A" else -0.35)
        e = max(rel(out[r].cpu().numpy(), A @ x[r].cpu().numpy()) for r in range(nrhs))
        say(f"noalloc {prec} {dims} nrhs {nrhs} {op}: equal to ovs_apply {same}, vs oracle {e:.1e}")
        assert same
        assert e <= (1e-14 if prec == "f64" else 1e-6)
        lat.close()


def test_noalloc_rejects_oversize():
    import paper_0810_4228_amd as ovs
    import torch
    dims = (16, 16, 16, 16)
    lat = _lattice(dims, "f64", 3, 0.2)
    x = torch.zeros((3, 12 * 16 ** 4), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(ovs.OvsError) as ei:   # 3 FP64 sources: 151 MB of staging > 64 MiB
        lat.apply_noalloc("A", x, out)
    assert ei.value.status == ovs.OVS_ERR_ARG
    lat.close()
