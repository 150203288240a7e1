"""GPU parity of the Wilson-Dirac stencil (Section 1) against the CPU oracle.

FP64: relative 2-norm error per source <= 1e-14; FP32 storage <= 1e-6
(single-precision rounding of links, inputs and accumulation).
"""
import numpy as np
import pytest

import synth
from oracle import dirac, freefield

from gpu_util import rel_rows, say, to_dev

pytestmark = pytest.mark.gpu

MW = -1.5
TOL = {"f64": 1e-14, "f32": 1e-6}


def lattice(dims, prec, U, mu):
    import paper_0810_4228_amd as ovs
    lat = ovs.Lattice(dims, precision=prec)
    lat.set_links(to_dev(U))
    lat.set_params(MW, mu)
    return lat


def oracle_op(dims, U, mu, op):
    if op in ("A", "A_dag"):
        m = dirac.csr_A(dims, U, MW, mu)
    else:
        m = dirac.csr_dw(dims, U, MW, mu)
    if op.endswith("dag"):
        m = m.conj().T.tocsr()
    return m


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 8, 10), (3, 2, 5, 4)])
@pytest.mark.parametrize("op", ["A", "A_dag", "Dw", "Dw_dag"])
def test_stencil_matches_csr(prec, dims, op):
    say("stencil", prec, dims, op)
    mu = 0.35
    U = synth.random_links(dims, 0.6, seed=3)
    b = synth.gaussian_sources(dims, 5, seed=4)
    lat = lattice(dims, prec, U, mu)
    y = lat.apply(op, to_dev(b)).cpu().numpy()
    ref = (oracle_op(dims, U, mu, op) @ b.T).T
    assert rel_rows(y, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 4, 7, 12])
def test_multi_rhs_blocks(prec, nrhs):
    """Every tuned source block gives the same result as the oracle (ragged tails)."""
    say("multi rhs", prec, nrhs)
    dims = (4, 4, 4, 8)
    U = synth.random_links(dims, 0.6, seed=5)
    b = synth.gaussian_sources(dims, nrhs, seed=6)
    lat = lattice(dims, prec, U, 0.2)
    lat.autotune(nrhs)
    y = lat.apply("A", to_dev(b)).cpu().numpy()
    ref = (oracle_op(dims, U, 0.2, "A") @ b.T).T
    assert rel_rows(y, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_stencil_configuration(prec):
    """Every stencil configuration the autotuner can pick (source block, lanes
    per site, LDS-staged tile, workgroup size, block order, streaming stores)
    against the oracle, for all four operators (the staged tile must apply
    gamma5 on input as the direct loads do): a ragged lattice (V = 576, not a
    multiple of any tile) and 7 sources (ragged source blocks)."""
    dims = (4, 4, 6, 6)
    mu = 0.3
    U = synth.random_links(dims, 0.6, seed=11)
    b = synth.gaussian_sources(dims, 7, seed=12)
    lat = lattice(dims, prec, U, mu)
    base = lat.get_tuning_raw(7)
    refs = {op: (oracle_op(dims, U, mu, op) @ b.T).T for op in ("A", "A_dag", "Dw", "Dw_dag")}
    shapes = [(blk, 1, st) for blk in ((1, 2, 3, 4, 6) if prec == "f32" else (1, 2, 3))
              for st in (0, 1) if st == 0 or blk <= (4 if prec == "f32" else 2)]
    shapes += [(1, g, 0) for g in (2, 4, 8)]
    n = 0
    for blk, g, st in shapes:
        for wg in (64, 128, 256):
            for order, nt in ((0, 0), (1, 1)):
                cfg = list(base)
                cfg[0:4] = [1000 * st + 100 * blk + 10 * g + nt, wg, 0, order]
                lat.set_tuning_raw(7, cfg)
                for op, ref in refs.items():
                    y = lat.apply(op, to_dev(b)).cpu().numpy()
                    e = rel_rows(y, ref)
                    assert e <= TOL[prec], (blk, g, st, wg, order, nt, op, e)
                n += 1
    say("stencil configurations", prec, n)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grouped_block_orders(prec):
    """Block orders 2-7 (each XCD sweeps its time chunk once per window of 1, 2,
    3, 4, 6 or all source blocks) need Lx Ly a multiple of the tile and Lt a
    multiple of 8:
    16 x 16 x 2 x 8 with 256-site tiles and 8 x 8 x 4 x 8 with 64-site tiles,
    7 sources (ragged windows), against the oracle."""
    for dims, wg in (((16, 16, 2, 8), 256), ((8, 8, 4, 8), 64)):
        U = synth.random_links(dims, 0.6, seed=13)
        b = synth.gaussian_sources(dims, 7, seed=14)
        lat = lattice(dims, prec, U, 0.3)
        base = lat.get_tuning_raw(7)
        ref = (oracle_op(dims, U, 0.3, "A") @ b.T).T
        blocks = (1, 2, 3) if prec == "f32" else (1, 2)
        for blk in blocks:
            for st in (0, 1):
                if st and blk > (4 if prec == "f32" else 2):
                    continue
                for order in range(2, 8):
                    cfg = list(base)
                    cfg[0:4] = [1000 * st + 100 * blk + 10 + 1, wg, 0, order]
                    lat.set_tuning_raw(7, cfg)
                    e = rel_rows(lat.apply("A", to_dev(b)).cpu().numpy(), ref)
                    assert e <= TOL[prec], (dims, blk, st, order, e)
        lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_links_from_host_memory(prec):
    """ovs_set_links with host links (on_device = 0) packs the same links as
    with device links: the operator's results are equal bit for bit."""
    import torch
    dims = (4, 4, 6, 8)
    U = synth.random_links(dims, 0.5, seed=17)
    x = to_dev(synth.gaussian_sources(dims, 3, seed=18))
    dev_lat = lattice(dims, prec, U, 0.25)
    import paper_0810_4228_amd as ovs
    host_lat = ovs.Lattice(dims, precision=prec)
    host_lat.set_links(U)   # numpy array: host memory
    host_lat.set_params(MW, 0.25)
    for op in ("A", "A_dag"):
        assert torch.equal(dev_lat.apply(op, x), host_lat.apply(op, x))
    dev_lat.close()
    host_lat.close()


def test_field_roundtrip_bitwise():
    import torch
    dims = (4, 4, 4, 4)
    U = synth.random_links(dims, 0.6, seed=7)
    lat = lattice(dims, "f64", U, 0.1)
    b = to_dev(synth.gaussian_sources(dims, 3, seed=8))
    f = lat.field_create(3)
    f.import_(b)
    out = f.export()
    assert torch.equal(out, b)


def test_field_apply_equals_apply():
    dims = (4, 4, 6, 8)
    U = synth.random_links(dims, 0.6, seed=9)
    lat = lattice(dims, "f32", U, 0.4)
    b = to_dev(synth.gaussian_sources(dims, 4, seed=10))
    fi, fo = lat.field_create(4), lat.field_create(4)
    fi.import_(b)
    fi.apply("A", fo)
    ms = fi.apply_timed("A", fo, 3)
    assert ms > 0
    y1 = fo.export().cpu().numpy()
    y2 = lat.apply("A", b).cpu().numpy()
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (16, 16, 16, 32)])
def test_full_size_sampled_sites(dims):
    """Full-size random links: sampled output sites against the per-site oracle."""
    say("sampled", dims)
    mu = 0.2
    U = synth.random_links(dims, 0.8, seed=0)
    b = synth.gaussian_sources(dims, 2, seed=1)
    for prec in ("f64", "f32"):
        lat = lattice(dims, prec, U, mu)
        lat.autotune(2)
        y = lat.apply("A", to_dev(b)).cpu().numpy().reshape(2, -1, 12)
        v = synth.volume(dims)
        rng = np.random.default_rng(5)
        sites = sorted(set(rng.integers(0, v, 40).tolist()) | {0, v - 1})
        for r in range(2):
            ref = dirac.apply_at_sites(dims, U, MW, mu, b[r], sites, op="A")
            err = np.linalg.norm(y[r][sites] - ref) / np.linalg.norm(ref)
            assert err <= TOL[prec] * 10, (prec, err)
        lat.close()


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (16, 16, 16, 32)])
def test_full_size_free_field(dims):
    """Unit links at full size: every output against the Fourier closed form."""
    say("free field", dims)
    mu = 0.4
    U = synth.unit_links(dims)
    b = synth.gaussian_sources(dims, 1, seed=2)
    ref = freefield.free_apply_A(dims, MW, mu, b)
    lat = lattice(dims, "f64", U, mu)
    y = lat.apply("A", to_dev(b)).cpu().numpy()
    assert rel_rows(y, ref) <= 1e-13


def test_gamma5_hermiticity_dot():
    """<u, A v> = <A(-mu) u, v> on the GPU operator itself."""
    dims = (4, 4, 4, 8)
    U = synth.random_links(dims, 0.6, seed=11)
    lat = lattice(dims, "f64", U, 0.3)
    u = synth.gaussian_sources(dims, 1, seed=12)[0]
    v = synth.gaussian_sources(dims, 1, seed=13)[0]
    Av = lat.apply("A", to_dev(v[None])).cpu().numpy()[0]
    Adu = lat.apply("A_dag", to_dev(u[None])).cpu().numpy()[0]
    lhs = np.vdot(u, Av)
    rhs = np.vdot(Adu, v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_dual_timed_entry_point():
    """ovs_dual_apply_timed: a positive time for a resident field that it leaves
    unchanged, and OVS_ERR_ARG for iters < 1 and for a field of another lattice."""
    import ctypes
    import paper_0810_4228_amd as ovs
    dims = (4, 4, 4, 8)
    U = synth.random_links(dims, 0.6, seed=21)
    b = synth.gaussian_sources(dims, 3, seed=22)
    lat = lattice(dims, "f32", U, 0.2)
    other = lattice(dims, "f32", U, 0.2)
    f = lat.field_create(3)
    f.import_(to_dev(b))
    before = f.export().cpu().numpy()
    assert f.dual_timed(5) > 0
    assert np.array_equal(f.export().cpu().numpy(), before)
    with pytest.raises(ovs.OvsError) as e:
        f.dual_timed(0)
    assert e.value.status == ovs.OVS_ERR_ARG
    g = other.field_create(3)
    ms = ctypes.c_double()
    assert lat._lib.ovs_dual_apply_timed(lat._h, g._h, 1, ctypes.byref(ms)) == ovs.OVS_ERR_ARG
    f.close()
    g.close()


def test_argument_errors():
    import paper_0810_4228_amd as ovs
    import torch
    with pytest.raises(ovs.OvsError):
        ovs.Lattice((1, 4, 4, 4))
    with pytest.raises(ovs.OvsError):
        ovs.Lattice((4, 4, 4, 4), bc=(1, 1, 1, 0))
    with pytest.raises(ovs.OvsError) as e:
        ovs.Lattice((64, 64, 64, 128))  # 2^25 sites: above the 2^24 limit
    assert e.value.status == ovs.OVS_ERR_ARG
    lat = ovs.Lattice((2, 2, 2, 2))
    x = torch.zeros((1, 12 * 16), dtype=torch.complex128, device="cuda")
    with pytest.raises(ovs.OvsError) as e:
        lat.apply("A", x)  # links not set
    assert e.value.status == ovs.OVS_ERR_STATE
    with pytest.raises(ovs.OvsError):
        lat.set_params(-4.0, 0.1)  # 8 + 2 m_w <= 0
