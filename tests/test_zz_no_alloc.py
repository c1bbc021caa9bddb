"""rhmc_apply_mdagm_static: A = m^2 - D_eo D_oe with its odd temporary and
partial sums in the library's static device scratch (no allocation), called
through the C ABI.  Its output must equal rhmc_apply_mdagm's bit for bit
(same kernels, same launch variants) on two calls in a row, the second with a
smaller input, and a call needing more than the 64 MiB of scratch must be
refused with INVALID_ARG and leave the output untouched."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rh():
    import torch

    from paper_1106_5673_amd import rhmc

    rhmc.load()
    assert torch.cuda.is_available()
    return rhmc


def _vec(rh, rng, prec, nrhs, Vh, dtype):
    """Random vector set in the ABI storage (even nrhs: the paired FP32 form
    holds as many entries as [nrhs][3][Vh])."""
    import torch

    v = rng.standard_normal((nrhs, 3, Vh)) + 1j * rng.standard_normal((nrhs, 3, Vh))
    return torch.from_numpy(v.astype(dtype).reshape(rh.vec_shape(prec, nrhs, Vh))).to("cuda:0")


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_static_mdagm_matches_mdagm(rh, prec_name):
    import torch

    prec = rh.RHMC_PREC_FP64 if prec_name == "fp64" else rh.RHMC_PREC_FP32
    dtype = np.complex128 if prec_name == "fp64" else np.complex64
    m = 0.03
    rng = np.random.default_rng(31)
    # first call: a larger lattice (staged launch shapes) and 4 rhs; second: a
    # smaller lattice and 1 rhs, reusing the scratch the first call left behind
    for L, nrhs, seed in (((16, 16, 8, 8), 4, 9100), ((8, 8, 4, 6), 1, 9101)):
        U = synth.gauge_field(L, 0.6, seed)
        lat = rh.rhmc_lattice_create(L, -1)
        g = rh.rhmc_gauge_create(lat, U)
        v = _vec(rh, rng, prec, nrhs, lat.Vh, dtype)
        ref = torch.empty_like(v)
        rh.rhmc_apply_mdagm(g, m, prec, nrhs, v, ref)
        for _ in range(2):
            out = torch.full_like(v, float("nan"))
            rh.rhmc_apply_mdagm_static(g, m, prec, nrhs, v, out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
        g.close()


def test_static_mdagm_refuses_oversize(rh):
    import torch

    # 48^3 x 12: 3 rhs in FP64 need 3 * 3 * 663552 * 16 B = 95.6 MB plus the
    # partial sums, above the 64 MiB of scratch (2 rhs, 64.4 MB, fit)
    L = (48, 48, 48, 12)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, synth.unit_gauge(L))
    v = torch.ones((3, 3, lat.Vh), dtype=torch.complex128, device="cuda:0")
    out = torch.zeros_like(v)
    with pytest.raises(rh.RhmcError) as e:
        rh.rhmc_apply_mdagm_static(g, 0.1, rh.RHMC_PREC_FP64, 3, v, out)
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    assert "64" in rh.rhmc_last_error() or "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    # two rhs fit and equal the allocating entry point
    ref = torch.empty_like(v[:2])
    rh.rhmc_apply_mdagm(g, 0.1, rh.RHMC_PREC_FP64, 2, v[:2], ref)
    got = torch.empty_like(ref)
    rh.rhmc_apply_mdagm_static(g, 0.1, rh.RHMC_PREC_FP64, 2, v[:2], got)
    assert torch.equal(got, ref)
    g.close()
