"""Parity of the HIP half hop and normal operator with the FP64 oracle.

FP64 kernels must agree to rounding (1e-13 relative to the largest entry);
FP32 kernels to 2e-6 (FP32 rounding of links and vectors over 8 hops)."""
import numpy as np
import pytest

from gpu_common import rel, to_dev, to_np, torch_gpu
from oracle import freefield as F
from oracle import oracle as O
from paper_1808_01829_amd.inputs import gaussian_block, random_gauge, unit_gauge

pytestmark = pytest.mark.gpu

CASES = [((2, 2, 2, 2), 1), ((4, 4, 4, 4), 1), ((4, 4, 4, 4), 16), ((4, 6, 2, 8), 3),
         ((8, 8, 8, 8), 4), ((2, 4, 6, 4), 5), ((8, 4, 4, 6), 8), ((4, 4, 4, 4), 32)]


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


def _ctx(dims, bc, U):
    from paper_1808_01829_amd import bms
    torch = torch_gpu()
    c = bms.Context(dims, bc)
    c.set_gauge(to_dev(torch, U))
    return c


@pytest.mark.parametrize("dims,n", CASES)
@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_hop_f64_and_f32(torch, dims, n, bc):
    from paper_1808_01829_amd import bms
    U = random_gauge(dims, 0.7, 101)
    c = _ctx(dims, bc, U)
    v = gaussian_block(dims, n, 102)
    # default kernel, then the one-thread-per-column-group kernel (variant 0)
    for variant in (-1, 0):
        c.set_variant(bms.BMS_KERNEL_HOP, variant)
        for par in (0, 1):
            ref = np.stack([O.dslash_half(dims, bc, U, par, v[..., j]) for j in range(n)], axis=-1)
            out = to_np(c.apply_hop(par, to_dev(torch, v)))
            assert rel(out, ref) < 1e-13
            out32 = to_np(c.apply_hop(par, to_dev(torch, v.astype(np.complex64)), bms.BMS_PREC_F32))
            assert rel(out32, ref) < 2e-6


@pytest.mark.parametrize("dims,n", CASES[:6])
def test_mdagm_f64_and_f32(torch, dims, n):
    from paper_1808_01829_amd import bms
    bc = (1, 1, 1, -1)
    U = random_gauge(dims, 0.9, 103)
    c = _ctx(dims, bc, U)
    v = gaussian_block(dims, n, 104)
    for sigma in (0.0, 0.75):
        ref = O.mdagm(dims, bc, U, 0.05, sigma, v)
        out = to_np(c.apply_mdagm(0.05, sigma, to_dev(torch, v)))
        assert rel(out, ref) < 1e-13
        out32 = to_np(c.apply_mdagm(0.05, sigma, to_dev(torch, v.astype(np.complex64)),
                                    bms.BMS_PREC_F32))
        assert rel(out32, ref) < 5e-6


def test_mdagm_full_size_sampled(torch):
    # 32^4 at n = 16 (the largest workload): columns 0 and 11 against the oracle
    dims, n, bc = (32, 32, 32, 32), 16, (1, 1, 1, -1)
    U = random_gauge(dims, 0.8, 5000)
    c = _ctx(dims, bc, U)
    v = gaussian_block(dims, n, 5001)
    out = to_np(c.apply_mdagm(0.01, 0.0, to_dev(torch, v)))
    for j in (0, 11):
        ref = O.mdagm(dims, bc, U, 0.01, 0.0, v[..., j])
        assert rel(out[..., j], ref) < 1e-13


def test_free_field_inverse_property(torch):
    # at U = 1, (A + s) applied to the exact FFT solution returns the source
    dims, n, bc = (16, 16, 16, 16), 4, (1, 1, 1, -1)
    c = _ctx(dims, bc, unit_gauge(dims))
    b = gaussian_block(dims, n, 7)
    x = F.solve(dims, bc, 0.02, 0.1, b)
    out = to_np(c.apply_mdagm(0.02, 0.1, to_dev(torch, x)))
    assert rel(out, b) < 1e-12


def test_errors(torch):
    from paper_1808_01829_amd import bms
    dims = (4, 4, 4, 4)
    c = bms.Context(dims)
    v = to_dev(torch, gaussian_block(dims, 2, 1))
    with pytest.raises(bms.BmsError) as e:
        c.apply_mdagm(0.1, 0.0, v)  # no gauge field yet
    assert e.value.code == bms.BMS_ESTATE
    c.set_gauge(to_dev(torch, unit_gauge(dims)))
    with pytest.raises(bms.BmsError) as e:
        bms.bms_apply_mdagm(c.h, 0.1, 0.0, 2, v, v)  # aliasing
    assert e.value.code == bms.BMS_EINVAL
    with pytest.raises(bms.BmsError) as e:
        bms.bms_apply_hop(c.h, 2, 2, v, torch.empty_like(v))
    assert e.value.code == bms.BMS_EINVAL


@pytest.mark.parametrize("n", [16, 8])
def test_hop_tiled_traversal(torch, n):
    # 16x16x32x4: the smallest lattice the 8x8x4-tile plan accepts (8 rows of
    # 8 checkerboard sites per work-group, (16/8)*(32/8) = 8 pencils, one per
    # XCD); every variant, natural and tiled, against the oracle
    from paper_1808_01829_amd import bms
    dims, bc = (16, 16, 32, 4), (1, 1, 1, -1)
    U = random_gauge(dims, 0.7, 105)
    c = _ctx(dims, bc, U)
    v = gaussian_block(dims, n, 106)
    aux = gaussian_block(dims, n, 107)
    for par in (0, 1):
        ref = np.stack([O.dslash_half(dims, bc, U, par, v[..., j]) for j in range(n)], axis=-1)
        for variant in (-1, 0, 1, 2, 3):
            c.set_variant(bms.BMS_KERNEL_HOP, variant)
            out = to_np(c.apply_hop(par, to_dev(torch, v)))
            assert rel(out, ref) < 1e-13, (par, variant)
            out32 = to_np(c.apply_hop(par, to_dev(torch, v.astype(np.complex64)), bms.BMS_PREC_F32))
            assert rel(out32, ref) < 2e-6, (par, variant)
    # the D_eo half hop with its aux term (M^dag M) through the tiled FP64 default
    for variant in (-1, 0, 3):
        c.set_variant(bms.BMS_KERNEL_HOP, variant)
        ref = O.mdagm(dims, bc, U, 0.05, 0.3, v)
        out = to_np(c.apply_mdagm(0.05, 0.3, to_dev(torch, v)))
        assert rel(out, ref) < 1e-13, variant


@pytest.mark.parametrize("dims,n", [((4, 4, 4, 4), 16), ((4, 6, 2, 8), 3), ((8, 4, 4, 6), 8)])
def test_hop_link_rows(torch, dims, n):
    """The hop reads SU(3) links as two rows and rebuilds the third: the same
    result as with all nine entries, both equal to the oracle; a field that is
    not SU(3) (one link off by 1e-9, or every link scaled) is read in full."""
    from paper_1808_01829_amd import bms
    bc = (1, 1, 1, -1)
    U = random_gauge(dims, 0.7, 105)
    v = gaussian_block(dims, n, 106)
    vd = to_dev(torch, v)
    c = _ctx(dims, bc, U)
    rows, dev = c.link_rows(with_deviation=True)
    print("link rows", rows, "third-row deviation", dev)
    assert rows == 2 and 0 <= dev <= 1e-14
    two = {}
    for par in (0, 1):
        ref = np.stack([O.dslash_half(dims, bc, U, par, v[..., j]) for j in range(n)], axis=-1)
        for variant in (-1, 0):
            c.set_variant(bms.BMS_KERNEL_HOP, variant)
            two[par, variant] = to_np(c.apply_hop(par, vd))
            assert rel(two[par, variant], ref) < 1e-13
            out32 = to_np(c.apply_hop(par, to_dev(torch, v.astype(np.complex64)), bms.BMS_PREC_F32))
            assert rel(out32, ref) < 2e-6
    c.set_variant(bms.BMS_KERNEL_HOP, -1)
    c.set_link_rows(3)
    c.set_gauge(to_dev(torch, U))
    assert c.link_rows() == 3
    for par in (0, 1):
        assert rel(to_np(c.apply_hop(par, vd)), two[par, -1]) < 1e-14
    with pytest.raises(bms.BmsError):
        c.set_link_rows(4)
    # fields the check turns away: one link perturbed, every link scaled
    c.set_link_rows(2)
    U1 = U.copy()
    U1[2, 5, 1, 2] += 1e-9
    U2 = U * 1.0001
    for Ub, lo in ((U1, 1e-10), (U2, 1e-5)):
        c.set_gauge(to_dev(torch, Ub))
        rows, dev = c.link_rows(with_deviation=True)
        assert rows == 3 and dev > lo
        for par in (0, 1):
            ref = np.stack([O.dslash_half(dims, bc, Ub, par, v[..., j]) for j in range(n)], axis=-1)
            assert rel(to_np(c.apply_hop(par, vd)), ref) < 1e-13
    c.set_gauge(to_dev(torch, U))
    assert c.link_rows() == 2
    c.close()


def test_link_form_follows_the_field(torch):
    """One context alternating between SU(3) links (read as two rows) and the
    improved operator's one-hop and three-hop links (nine entries, not SU(3)):
    each hop equals the oracle's for the field loaded last."""
    from paper_1808_01829_amd import bms
    dims, n, bc = (4, 4, 6, 4), 4, (1, 1, 1, -1)
    U = random_gauge(dims, 0.6, 107)
    V, W = U * (9.0 / 8.0), random_gauge(dims, 0.6, 108) * (-1.0 / 24.0)
    v = gaussian_block(dims, n, 109)
    vd = to_dev(torch, v)
    c = _ctx(dims, bc, U)
    for step in range(3):
        improved = step == 1
        if improved:
            c.set_gauge_improved(to_dev(torch, V), to_dev(torch, W))
        elif step == 2:
            c.set_gauge(to_dev(torch, U))
        rows, dev = c.link_rows(with_deviation=True)
        assert rows == (3 if improved else 2)
        assert (dev == -1.0) if improved else (0 <= dev <= 1e-14)
        for par in (0, 1):
            if improved:
                ref = np.stack([O.dslash_half(dims, bc, V, par, v[..., j], W) for j in range(n)], -1)
            else:
                ref = np.stack([O.dslash_half(dims, bc, U, par, v[..., j]) for j in range(n)], -1)
            assert rel(to_np(c.apply_hop(par, vd)), ref) < 1e-13
    c.close()


def test_hop_streamed(torch):
    """The streamed half hop (variant 4, n = 16: persistent waves, the next
    hops' columns and links in flight through a ring in LDS) against the
    oracle: tiled and natural traversals, ring depths 2 and 4, with and
    without the non-temporal link hint, FP64 and FP32, two-row and nine-entry
    SU(3) links and the improved operator, the D_eo hop with its aux term,
    and lattices it does not take (another kernel runs)."""
    from paper_1808_01829_amd import bms
    dims, bc, n = (16, 16, 32, 4), (1, 1, 1, -1), 16
    U = random_gauge(dims, 0.7, 111)
    v = gaussian_block(dims, n, 112)
    vd, v32 = to_dev(torch, v), to_dev(torch, v.astype(np.complex64))
    ref = {par: np.stack([O.dslash_half(dims, bc, U, par, v[..., j]) for j in range(n)], axis=-1)
           for par in (0, 1)}
    mref = O.mdagm(dims, bc, U, 0.05, 0.3, v)
    c = _ctx(dims, bc, U)
    c.set_variant(bms.BMS_KERNEL_HOP, 4)
    cfgs = [None, (8, 8, 4, 2, 1), (8, 8, 4, 4, 0), (0, 0, 0, 2, 0), (0, 0, 0, 4, 1), (16, 8, 4, 4, 1)]
    for rows in (2, 3):
        c.set_link_rows(rows)
        c.set_gauge(to_dev(torch, U))
        assert c.link_rows() == rows
        for cfg in cfgs:
            for prec in (bms.BMS_PREC_F64, bms.BMS_PREC_F32):
                c.set_hop_config(prec, cfg)
            for par in (0, 1):
                out = to_np(c.apply_hop(par, vd))
                assert rel(out, ref[par]) < 1e-13, (rows, cfg, par)
                out32 = to_np(c.apply_hop(par, v32, bms.BMS_PREC_F32))
                assert rel(out32, ref[par]) < 2e-6, (rows, cfg, par)
            assert rel(to_np(c.apply_mdagm(0.05, 0.3, vd)), mref) < 1e-13, (rows, cfg)
            m32 = to_np(c.apply_mdagm(0.05, 0.3, v32, bms.BMS_PREC_F32))
            assert rel(m32, mref) < 2e-6, (rows, cfg)
    # the improved operator (16 links per site)
    V = random_gauge(dims, 0.7, 113) * (9.0 / 8.0)
    W = random_gauge(dims, 0.7, 114) * (-1.0 / 24.0)
    c.set_gauge_improved(to_dev(torch, V), to_dev(torch, W))
    for cfg in (None, (0, 0, 0, 2, 1)):
        for prec in (bms.BMS_PREC_F64, bms.BMS_PREC_F32):
            c.set_hop_config(prec, cfg)
        for par in (0, 1):
            r = np.stack([O.dslash_half(dims, bc, V, par, v[..., j], W) for j in range(n)], axis=-1)
            assert rel(to_np(c.apply_hop(par, vd)), r) < 1e-13, (cfg, par)
            assert rel(to_np(c.apply_hop(par, v32, bms.BMS_PREC_F32)), r) < 2e-6, (cfg, par)
    c.close()
    # lattices the streamed kernel does not take (V/2 not a multiple of 128,
    # n != 16) run another kernel with the same result
    for dims2, n2 in (((4, 6, 2, 8), 16), ((8, 8, 8, 8), 8)):
        U2 = random_gauge(dims2, 0.7, 115)
        v2 = gaussian_block(dims2, n2, 116)
        c2 = _ctx(dims2, bc, U2)
        c2.set_variant(bms.BMS_KERNEL_HOP, 4)
        for par in (0, 1):
            r = np.stack([O.dslash_half(dims2, bc, U2, par, v2[..., j]) for j in range(n2)], axis=-1)
            assert rel(to_np(c2.apply_hop(par, to_dev(torch, v2))), r) < 1e-13, (dims2, par)
        c2.close()
