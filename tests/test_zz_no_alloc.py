"""gpe_apply_h_noalloc (the entry point for callers that cannot allocate)
against gpe_apply_h, through the C ABI: the same H(phi)phi and scalars on two
calls in a row (the second on a smaller grid, so the fixed scratch holds the
first call's contents), in both precisions, and the size limit."""
import ctypes as C
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ("energy", "mu", "resid", "norm2", "rms_x", "rms_y", "rms_z", "max_dens", "e_kin", "e_pot")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_02891_amd import api
    return api


def _field(p, seed):
    rng = np.random.default_rng(seed)
    cs = disc.grid_coords(p)
    r2 = sum(c * c for c in cs)
    phi = np.exp(-r2 / 4.0) * (1 + 0.5j * cs[0]) + 0.05 * (rng.standard_normal(p.shape)
                                                           + 1j * rng.standard_normal(p.shape))
    return phi / math.sqrt(disc.h_vol(p) * float(np.sum(np.abs(phi) ** 2)))


def _bound(p, phi, prec):
    """Rounding bound of one application of H (as in the primitive tests)."""
    eps, cf = (2.0 ** -53, 16.0) if prec == "fp64" else (2.0 ** -24, 32.0)
    lam = [math.pi * p.n[a] / (p.hi[a] - p.lo[a]) for a in range(p.dim)]
    rot = max(abs(p.omega) * max(abs(p.lo[b]), abs(p.hi[b])) for b in range(p.dim)) if p.dim > 1 else 0.0
    mult = sum(0.5 * l * l + rot * l for l in lam)
    amax = float(np.max(np.abs(phi)))
    lg = max(math.log2(n) for n in p.n)
    return cf * eps * lg * (mult + float(np.max(disc.potential(p))) + p.beta * amax ** 2) * amax


CASES = [
    W.Problem(dim=3, n=(128, 64, 64), lo=(-12.0, -8.0, -8.0), hi=(12.0, 8.0, 8.0), beta=800.0,
              omega=0.3, lattice_amp=20.0),
    W.Problem(dim=2, n=(64, 32), lo=(-8.0, -6.0), hi=(8.0, 6.0), beta=300.0, omega=0.7),
]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_apply_h_on_two_calls(dev, prec):
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    for k, p in enumerate(CASES):           # the second grid is smaller than the first
        print(f"noalloc {prec} case {k} n={p.n}", flush=True)
        t = torch.from_numpy(_field(p, 3 + k)).to(dt).cuda()
        ref, sc = dev.apply_h(p, t, precision=prec)
        sd = torch.full((10,), float("nan"), dtype=torch.float64, device="cuda")
        got = dev.apply_h_noalloc(p, t, precision=prec, scalars_out=sd)
        torch.cuda.synchronize()
        g = got.cpu().numpy().astype(np.complex128)
        r = ref.cpu().numpy().astype(np.complex128)
        phi_in = t.cpu().numpy().astype(np.complex128)
        # the same kernels: the outputs agree to the last bits of V
        # (the tables are evaluated on the device here, on the host there)
        same = (1e-13 if prec == "fp64" else 2.0 ** -21) * float(np.max(np.abs(r)))
        assert float(np.max(np.abs(g - r))) <= same
        # and both are H(phi)phi of the oracle to the rounding bound
        ora = disc.h_full(p, phi_in)
        assert float(np.max(np.abs(g - ora))) <= _bound(p, phi_in, prec)
        s = sd.cpu().numpy()
        rt = 1e-12 if prec == "fp64" else 1e-6
        for i, name in enumerate(NAMES):
            if name == "rms_z" and p.dim < 3:
                continue
            assert abs(s[i] - sc[name]) <= rt * abs(sc[name]) + 1e-14, (name, s[i], sc[name])


def test_noalloc_without_scalars_and_size_limit(dev):
    from paper_1504_02891_amd import _native as N
    p = CASES[1]
    t = torch.from_numpy(_field(p, 9)).cuda()
    ref, _ = dev.apply_h(p, t)
    got = dev.apply_h_noalloc(p, t)
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(got - ref))) <= 1e-13 * float(torch.max(torch.abs(ref)))
    # above the scratch's 2^21 points: refused before any device work
    big = W.Problem(dim=3, n=(256, 128, 128), lo=(-8.0,) * 3, hi=(8.0,) * 3, beta=1.0)
    ps = dev.problem_struct(big)
    rc = N.lib().gpe_apply_h_noalloc(dev.context(0), C.byref(ps), N.GPE_PREC_FP64, C.c_void_p(t.data_ptr()),
                                     C.c_void_p(got.data_ptr()), None)
    assert rc == N.GPE_EUNSUPPORTED
    assert b"exceed" in N.lib().gpe_last_error()
