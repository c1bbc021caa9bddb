"""GPU parity of the hopping term, A = m^2 - D_eo D_oe and the neighbour tables.

Everything goes through the C ABI (ctypes binding) and is compared with the
FP64 CPU oracle on the same seeded inputs:
  * neighbour indices and hop signs: bit-exact;
  * point sources on unit links: bit-exact (single products of +-1/2);
  * random SU(3) fields, FP64 path: max |gpu - oracle| <= 1e-13 * max |oracle|,
    well inside the 1e-12 relative budget (FMA contraction and summation order
    differ, each output is a sum of 24 products);
  * FP32 path with 12-real links: |gpu - oracle| <= 32 * 2^-24 * scale per
    element, scale = 1/2 sum over the 8 hops of |U| |psi| (rounding of links,
    vectors, the third-row rebuild and 24 accumulations).
FP32 sets of two or more right-hand sides are passed in the ABI's paired
storage (f32layout).
"""

import numpy as np
import pytest

import dslash_bound
import f32layout
import synth
from oracle import dirac, lattice

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (2, 4, 6, 8), (6, 2, 4, 2), (8, 8, 8, 6), (16, 16, 16, 4)]


@pytest.fixture(scope="module")
def rh():
    import torch

    from paper_1106_5673_amd import rhmc

    rhmc.load()
    assert torch.cuda.is_available()
    return rhmc


def _dev():
    import torch

    return torch.device("cuda:0")


def _to(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _rand_vec(rng, nrhs, Vh):
    return (rng.standard_normal((nrhs, 3, Vh)) + 1j * rng.standard_normal((nrhs, 3, Vh)))


@pytest.mark.parametrize("L", LATTICES + [(2, 2, 2, 2)])
@pytest.mark.parametrize("t_bc", [-1, 1])
def test_neighbors_bit_exact(rh, L, t_bc):
    lat = rh.rhmc_lattice_create(L, t_bc)
    for par in (0, 1):
        nb, sg = rh.rhmc_debug_neighbors(lat, par)
        assert np.array_equal(nb, lattice.neighbor_table(L, par))
        x, y, z, t = lattice.eo_coordinates(L, par)
        bc = lattice.boundary_sign_table(L, par, t_bc)
        eta = np.stack([np.ones_like(x), (-1) ** x, (-1) ** (x + y), (-1) ** (x + y + z)], axis=1)
        expect = np.concatenate([eta, eta], axis=1) * bc
        assert np.array_equal(sg, expect)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_point_sources_unit_links_bit_exact(rh, prec):
    import torch

    L = (4, 4, 4, 4)
    U = synth.unit_gauge(L)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    Vh = lat.Vh
    p = rh.RHMC_PREC_FP64 if prec == "fp64" else rh.RHMC_PREC_FP32
    cdt = np.complex128 if prec == "fp64" else np.complex64
    srcs = [(0, 0, 5), (1, 2, 77), (2, 1, 127), (0, 0, 0)]
    for out_par in (0, 1):
        v = np.zeros((len(srcs), 3, Vh), dtype=cdt)
        for k, (c, _, eo) in enumerate(srcs):
            v[k, c, eo] = 1.0
        vin = _to(v if prec == "fp64" else f32layout.pack(v))
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, p, len(srcs), vin, vout)
        torch.cuda.synchronize()
        ref = dirac.dslash(U, v.astype(np.complex128), out_par)
        got = vout.cpu().numpy()
        if prec == "fp32":
            got = f32layout.unpack(got, len(srcs), Vh)
        assert np.array_equal(got.astype(np.complex128), ref)
    g.close()


_abs_scale = dslash_bound.abs_scale


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_dslash_random_fields(rh, L, nrhs):
    import torch

    t_bc = -1
    U = synth.gauge_field(L, 0.7, 4000 + sum(L))
    lat = rh.rhmc_lattice_create(L, t_bc)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(11)
    for out_par in (0, 1):
        v = _rand_vec(rng, nrhs, lat.Vh)
        ref = dirac.dslash(U, v, out_par, t_bc)
        vin = _to(v)
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP64, nrhs, vin, vout)
        torch.cuda.synchronize()
        got = vout.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
        # FP32 with 12-real links
        v32 = v.astype(np.complex64)
        ref32 = dirac.dslash(U, v32.astype(np.complex128), out_par, t_bc)
        vin = _to(f32layout.pack(v32))
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP32, nrhs, vin, vout)
        torch.cuda.synchronize()
        got32 = f32layout.unpack(vout.cpu().numpy(), nrhs, lat.Vh).astype(np.complex128)
        scale = _abs_scale(U, v32.astype(np.complex128), out_par)
        err = np.abs(got32 - ref32)
        assert np.all(err.real <= 32 * 2.0 ** -24 * scale + 1e-30)
    g.close()


@pytest.mark.parametrize("nrhs", [2, 8, 11])
def test_multi_rhs_matches_single(rh, nrhs):
    """Batched right-hand sides give the same answer as one at a time."""
    import torch

    L = (8, 8, 8, 6)
    U = synth.gauge_field(L, 0.7, 4100)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(12)
    v = _rand_vec(rng, nrhs, lat.Vh)
    for prec, cdt in ((rh.RHMC_PREC_FP64, np.complex128), (rh.RHMC_PREC_FP32, np.complex64)):
        vc = v.astype(cdt)
        vin = _to(vc if cdt == np.complex128 else f32layout.pack(vc))
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, 0, prec, nrhs, vin, vout)
        torch.cuda.synchronize()
        got = vout.cpu().numpy()
        if cdt == np.complex64:
            got = f32layout.unpack(got, nrhs, lat.Vh)
        one = torch.empty((1, 3, lat.Vh), dtype=vin.dtype, device=_dev())
        for r in range(nrhs):
            rh.rhmc_dslash_eo(g, 0, prec, 1, _to(vc[r:r + 1]), one)
            torch.cuda.synchronize()
            # the same arithmetic per site and rhs: identical bits
            assert np.array_equal(got[r], one[0].cpu().numpy()), (prec, r)
    g.close()


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (16, 16, 16, 4)])
def test_mdagm_matches_oracle(rh, L):
    import torch

    m = 0.02
    U = synth.gauge_field(L, 0.5, 4200)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(13)
    v = _rand_vec(rng, 2, lat.Vh)
    ref = dirac.mdagm(U, m, v)
    vin = _to(v)
    vout = torch.empty_like(vin)
    rh.rhmc_apply_mdagm(g, m, rh.RHMC_PREC_FP64, 2, vin, vout)
    torch.cuda.synchronize()
    got = vout.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    vin32 = _to(f32layout.pack(v.astype(np.complex64)))
    vout32 = torch.empty_like(vin32)
    rh.rhmc_apply_mdagm(g, m, rh.RHMC_PREC_FP32, 2, vin32, vout32)
    torch.cuda.synchronize()
    got32 = f32layout.unpack(vout32.cpu().numpy(), 2, lat.Vh).astype(np.complex128)
    assert np.linalg.norm(got32 - ref) <= 1e-5 * np.linalg.norm(ref)
    g.close()


def test_invalid_arguments(rh):
    import torch

    with pytest.raises(rh.RhmcError) as e:
        rh.rhmc_lattice_create((4, 4, 3, 4))
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    L = (4, 4, 4, 4)
    lat = rh.rhmc_lattice_create(L)
    g = rh.rhmc_gauge_create(lat, synth.unit_gauge(L), flags=rh.RHMC_LINKS_FP64_18)
    v = torch.zeros((1, 3, lat.Vh), dtype=torch.complex64, device=_dev())
    with pytest.raises(rh.RhmcError) as e:
        rh.rhmc_dslash_eo(g, 0, rh.RHMC_PREC_FP32, 1, v, torch.empty_like(v))
    assert e.value.status == rh.RHMC_ERR_INVALID_ARG
    g.close()


@pytest.mark.parametrize("L", [(4, 6, 8, 4), (6, 4, 6, 8), (16, 8, 4, 6), (32, 8, 6, 4)])
def test_every_launch_variant_gives_identical_bits(rh, L):
    """All 192 launch variants (site order, load batching, block shape with or
    without rows staged in LDS, rhs tile)
    compute every output site with the same arithmetic: D_eo, D_oe and A agree
    bit for bit with variant 0, which is checked against the oracle.  z-tiles
    that do not divide Lz exercise the fallback; the last two lattices admit
    staged blocks (64 sites of 8 rows; 64 and 128 sites of 4 and 8 rows) whose
    periodic y halo and x wrap then come from LDS."""
    import torch

    t_bc = -1
    m = 0.05
    U = synth.gauge_field(L, 0.7, 4300 + sum(L))
    lat = rh.rhmc_lattice_create(L, t_bc)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(14)
    for prec, cdt in ((rh.RHMC_PREC_FP64, np.complex128), (rh.RHMC_PREC_FP32, np.complex64)):
        f32 = cdt == np.complex64
        for nrhs in (1, 3, 8):
            v = _rand_vec(rng, nrhs, lat.Vh).astype(cdt)
            vin = _to(f32layout.pack(v) if f32 else v)
            ref = {}
            for var in range(192):
                rh.rhmc_set_dslash_variant(g, prec, nrhs, var)
                assert rh.rhmc_dslash_variant(g, prec, nrhs) == var
                for out_par in (0, 1):
                    vout = torch.empty_like(vin)
                    rh.rhmc_dslash_eo(g, out_par, prec, nrhs, vin, vout)
                    got = vout.cpu().numpy()
                    if f32:
                        got = f32layout.unpack(got, nrhs, lat.Vh)
                    if var == 0:
                        ref[out_par] = got
                        v64 = v.astype(np.complex128)
                        want = dirac.dslash(U, v64, out_par, t_bc)
                        if cdt == np.complex128:
                            assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
                        else:
                            err = np.abs(got.astype(np.complex128) - want)
                            assert np.all(err <= 32 * 2.0 ** -24 * _abs_scale(U, v64, out_par) + 1e-30)
                    else:
                        assert np.array_equal(got, ref[out_par]), (var, out_par)
                vA = torch.empty_like(vin)
                rh.rhmc_apply_mdagm(g, m, prec, nrhs, vin, vA)
                gotA = vA.cpu().numpy()
                if f32:
                    gotA = f32layout.unpack(gotA, nrhs, lat.Vh)
                if var == 0:
                    ref["A"] = gotA
                else:
                    assert np.array_equal(gotA, ref["A"]), (var, "A")
    with pytest.raises(rh.RhmcError):
        rh.rhmc_set_dslash_variant(g, rh.RHMC_PREC_FP64, 1, 192)
    g.close()


def test_hilo_links_fp64_operator(rh):
    """hi/lo split (Sec. 4.2): the FP64 operator rebuilt from two FP32-12 planes
    agrees with the oracle to 1e-13 and with the FP64-18 operator to ~2^-45
    relative; the FP32 operator (hi only) is unchanged bit for bit."""
    import torch

    L = (8, 8, 8, 6)
    t_bc = -1
    U = synth.gauge_field(L, 0.7, 4400)
    lat = rh.rhmc_lattice_create(L, t_bc)
    g18 = rh.rhmc_gauge_create(lat, U)
    ghl = rh.rhmc_gauge_create(lat, U, flags=rh.RHMC_LINKS_HILO_12)
    rng = np.random.default_rng(15)
    v = _rand_vec(rng, 3, lat.Vh)
    for out_par in (0, 1):
        vin = _to(v)
        o18, ohl = torch.empty_like(vin), torch.empty_like(vin)
        rh.rhmc_dslash_eo(g18, out_par, rh.RHMC_PREC_FP64, 3, vin, o18)
        rh.rhmc_dslash_eo(ghl, out_par, rh.RHMC_PREC_FP64, 3, vin, ohl)
        want = dirac.dslash(U, v, out_par, t_bc)
        got = ohl.cpu().numpy()
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= 1e-13 * scale
        assert np.abs(got - o18.cpu().numpy()).max() <= 2.0 ** -45 * scale
        v32 = _to(f32layout.pack(v.astype(np.complex64)))
        a32, b32 = torch.empty_like(v32), torch.empty_like(v32)
        rh.rhmc_dslash_eo(g18, out_par, rh.RHMC_PREC_FP32, 3, v32, a32)
        rh.rhmc_dslash_eo(ghl, out_par, rh.RHMC_PREC_FP32, 3, v32, b32)
        assert np.array_equal(f32layout.unpack(a32.cpu().numpy(), 3, lat.Vh),
                              f32layout.unpack(b32.cpu().numpy(), 3, lat.Vh))
    g18.close()
    ghl.close()


def test_fp64_12_links_and_su3_check(rh):
    """FP64-12 storage (rows 1-2, row 3 rebuilt in FP64) gives the FP64-18
    operator to rounding; links that are not SU(3) to 1e-12 are refused for
    it (and default storage falls back to FP64-18), and links far from SU(3)
    are refused for the 12-real FP32 copy (default storage: FP32-18)."""
    import torch

    L = (6, 4, 4, 8)
    U = synth.gauge_field(L, 0.7, 4500)
    lat = rh.rhmc_lattice_create(L, -1)
    g12 = rh.rhmc_gauge_create(lat, U, flags=rh.RHMC_LINKS_FP64_12)
    g18 = rh.rhmc_gauge_create(lat, U, flags=rh.RHMC_LINKS_FP64_18)
    rng = np.random.default_rng(16)
    v = _rand_vec(rng, 2, lat.Vh)
    vin = _to(v)
    a, b = torch.empty_like(vin), torch.empty_like(vin)
    rh.rhmc_dslash_eo(g12, 1, rh.RHMC_PREC_FP64, 2, vin, a)
    rh.rhmc_dslash_eo(g18, 1, rh.RHMC_PREC_FP64, 2, vin, b)
    want = dirac.dslash(U, v, 1, -1)
    scale = np.abs(want).max()
    assert np.abs(a.cpu().numpy() - want).max() <= 1e-13 * scale
    assert np.abs(a.cpu().numpy() - b.cpu().numpy()).max() <= 1e-14 * scale
    with pytest.raises(rh.RhmcError):   # FP64-12 has no FP32 copy
        rh.rhmc_dslash_eo(g12, 1, rh.RHMC_PREC_FP32, 1, vin[:1].to(torch.complex64).contiguous(),
                          torch.empty((1, 3, lat.Vh), dtype=torch.complex64, device="cuda:0"))
    g12.close()
    g18.close()
    # row 3 off by 1e-9: no FP64-12, default storage falls back to FP64-18
    Ub = np.array(U)
    Ub[..., 2, :] *= 1 + 1e-9
    with pytest.raises(rh.RhmcError):
        rh.rhmc_gauge_create(lat, Ub, flags=rh.RHMC_LINKS_FP64_12)
    gb = rh.rhmc_gauge_create(lat, Ub)
    out = torch.empty_like(vin)
    rh.rhmc_dslash_eo(gb, 1, rh.RHMC_PREC_FP64, 2, vin, out)
    wantb = dirac.dslash(Ub, v, 1, -1)
    assert np.abs(out.cpu().numpy() - wantb).max() <= 1e-13 * np.abs(wantb).max()
    gb.close()
    # far from SU(3): refused for 12-real FP32 storage; the default storage is
    # then FP32-18 + FP64-18
    Uc = np.array(U)
    Uc[..., 2, :] *= 1.01
    with pytest.raises(rh.RhmcError):
        rh.rhmc_gauge_create(lat, Uc, flags=rh.RHMC_LINKS_FP32_12 | rh.RHMC_LINKS_FP64_18)
    rh.rhmc_gauge_create(lat, Uc, flags=rh.RHMC_LINKS_FP64_18).close()
    gc = rh.rhmc_gauge_create(lat, Uc)
    v32 = vin[:1].to(torch.complex64).contiguous()
    o32 = torch.empty_like(v32)
    rh.rhmc_dslash_eo(gc, 1, rh.RHMC_PREC_FP32, 1, v32, o32)
    wantc = dirac.dslash(Uc, v32.cpu().numpy().astype(np.complex128), 1, -1)
    assert np.abs(o32.cpu().numpy() - wantc).max() <= 1e-5 * np.abs(wantc).max()
    gc.close()


def test_max_rhs_and_direct_tuning(rh):
    """64 right-hand sides in one call (eight launches of eight) equal
    one-at-a-time results to FP64 rounding, and rhmc_tune_dslash picks a valid
    variant without changing any result bit."""
    import torch

    L = (4, 4, 4, 6)
    U = synth.gauge_field(L, 0.6, 4600)
    lat = rh.rhmc_lattice_create(L, -1)
    g = rh.rhmc_gauge_create(lat, U)
    rng = np.random.default_rng(17)
    v = _to(_rand_vec(rng, 64, lat.Vh))
    out = torch.empty_like(v)
    rh.rhmc_dslash_eo(g, 0, rh.RHMC_PREC_FP64, 64, v, out)
    one = torch.empty_like(v[:1])
    for r in (0, 7, 8, 63):
        rh.rhmc_dslash_eo(g, 0, rh.RHMC_PREC_FP64, 1, v[r:r + 1].contiguous(), one)
        assert (one[0] - out[r]).abs().max().item() <= 1e-15 * one.abs().max().item()
    v32 = _to(f32layout.pack(v[:4].cpu().numpy().astype(np.complex64)))
    a, b = torch.empty_like(v32), torch.empty_like(v32)
    rh.rhmc_dslash_eo(g, 1, rh.RHMC_PREC_FP32, 4, v32, a)
    rh.rhmc_tune_dslash(g, rh.RHMC_PREC_FP32, 4, v32, b)
    var = rh.rhmc_dslash_variant(g, rh.RHMC_PREC_FP32, 4)
    assert 0 <= var < 192
    rh.rhmc_dslash_eo(g, 1, rh.RHMC_PREC_FP32, 4, v32, b)
    assert torch.equal(a, b)
    g.close()


def _non_su3_links(L, seed):
    """Links that are not SU(3) (an SU(3) field plus 0.3 x complex noise): the
    staggered D stays anti-Hermitian for any links, so A stays Hermitian."""
    U = synth.gauge_field(L, 0.6, seed)
    rng = np.random.default_rng(seed + 1)
    return U + 0.3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))


@pytest.mark.parametrize("su3", [True, False])
@pytest.mark.parametrize("nrhs", [1, 4])
def test_fp32_18_links(rh, su3, nrhs):
    """FP32-18 storage: the FP32 operator from all 18 reals (no reconstruction),
    within the FP32 rounding bound of the oracle for SU(3) links and for links
    that are not SU(3) (which 12-real storage refuses); the default flags
    choose FP32-18 and FP64-18 for the latter; launch variants give the same bits."""
    import torch

    L = (6, 4, 4, 8)
    U = synth.gauge_field(L, 0.7, 4100) if su3 else _non_su3_links(L, 4100)
    lat = rh.rhmc_lattice_create(L, -1)
    flags = rh.RHMC_LINKS_FP32_18 | rh.RHMC_LINKS_FP64_18 if su3 else 0
    g = rh.rhmc_gauge_create(lat, U, flags)
    if not su3:
        with pytest.raises(rh.RhmcError):
            rh.rhmc_gauge_create(lat, U, rh.RHMC_LINKS_FP32_12 | rh.RHMC_LINKS_FP64_18)
    rng = np.random.default_rng(12)
    for out_par in (0, 1):
        v32 = _rand_vec(rng, nrhs, lat.Vh).astype(np.complex64)
        v = v32.astype(np.complex128)
        ref = dirac.dslash(U, v, out_par, -1)
        vin = _to(f32layout.pack(v32))
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP32, nrhs, vin, vout)
        torch.cuda.synchronize()
        got = f32layout.unpack(vout.cpu().numpy(), nrhs, lat.Vh).astype(np.complex128)
        scale = _abs_scale(U, v, out_par)
        err = np.abs(got - ref)
        assert np.all(err.real <= 32 * 2.0 ** -24 * scale + 1e-30)
        # the FP64 operator on the same gauge object
        vin64 = _to(v)
        vout64 = torch.empty_like(vin64)
        rh.rhmc_dslash_eo(g, out_par, rh.RHMC_PREC_FP64, nrhs, vin64, vout64)
        torch.cuda.synchronize()
        assert np.abs(vout64.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    # every launch variant computes the same bits
    outs = []
    for var in (0, 14, 36, 44, 71):
        rh.rhmc_set_dslash_variant(g, rh.RHMC_PREC_FP32, nrhs, var)
        vout = torch.empty_like(vin)
        rh.rhmc_dslash_eo(g, 1, rh.RHMC_PREC_FP32, nrhs, vin, vout)
        torch.cuda.synchronize()
        outs.append(vout.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    g.close()
