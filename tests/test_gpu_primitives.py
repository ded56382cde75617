"""GPU parity of the primitives (H(phi)phi, Hessian-vector product, Cayley
retraction, prolongation) against the oracle, through the C ABI.

Tolerance of a spectral pass (rounding analysis of a radix-2^k FFT pair):
|err| <= C * eps * log2(N) * (max|multiplier| + max|V| + beta max|phi|^2) * max|phi|,
with eps the unit roundoff of the transform precision and C = 4 in both
precisions; reductions accumulate in FP64.  Measured on MI355X the worst
error is about 0.024 of this bound in both precisions (H(phi)phi; the FP32
Hessian-vector product about 0.016): each test prints its ratio.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc
from oracle.cascade import prolong_fourier
from oracle.feasible import cayley_coefficients
from oracle.unified import UnifiedProblem, re_dot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = {"fp64": 2.0 ** -53, "mixed": 2.0 ** -24}
CFAC = {"fp64": 4.0, "mixed": 4.0}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_02891_amd import api
    return api


def _bound(p, phi, prec):
    """Rounding bound of one application of H (see the module docstring)."""
    lam = [math.pi * p.n[a] / (p.hi[a] - p.lo[a]) for a in range(p.dim)]
    rot = max(abs(p.omega) * max(abs(p.lo[b]), abs(p.hi[b])) for b in range(p.dim)) if p.dim > 1 else 0.0
    mult = sum(0.5 * l * l + rot * l for l in lam)
    vmax = float(np.max(disc.potential(p)))
    amax = float(np.max(np.abs(phi)))
    # transform length: n (Fourier) or the 2n-point odd extension (sine)
    lg = max(math.log2(2 * n if p.bc == W.SINE else n) for n in p.n)
    return CFAC[prec] * EPS[prec] * lg * (mult + vmax + p.beta * amax ** 2) * amax


def _field(p, seed):
    rng = np.random.default_rng(seed)
    cs = disc.grid_coords(p)
    r2 = sum(c * c for c in cs)
    smooth = np.exp(-r2 / 4.0) * (1 + 0.5j * cs[0])
    noise = 0.05 * (rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape))
    phi = smooth + noise
    return phi / math.sqrt(disc.h_vol(p) * float(np.sum(np.abs(phi) ** 2)))


CASES = [
    W.Problem(dim=1, n=(16,), lo=(-4.0,), hi=(4.0,), beta=10.0),
    W.Problem(dim=1, n=(512,), lo=(-16.0,), hi=(16.0,), beta=400.0),
    W.Problem(dim=1, n=(1024,), lo=(-20.0,), hi=(20.0,), beta=50.0, lattice_amp=25.0),
    W.Problem(dim=2, n=(64, 32), lo=(-8.0, -6.0), hi=(8.0, 6.0), beta=300.0, omega=0.7),
    W.Problem(dim=2, n=(16, 1024), lo=(-5.0, -20.0), hi=(5.0, 20.0), beta=100.0, omega=0.3),
    W.Problem(dim=2, n=(256, 256), lo=(-12.0, -12.0), hi=(12.0, 12.0), beta=1000.0, omega=0.9),
    W.Problem(dim=3, n=(32, 16, 64), lo=(-6.0, -5.0, -7.0), hi=(6.0, 5.0, 7.0), beta=200.0,
              omega=0.4, gamma=(1.0, 1.5, 2.0), lattice_amp=10.0),
    W.Problem(dim=3, n=(128, 128, 128), lo=(-16.0,) * 3, hi=(16.0,) * 3, beta=1600.0,
              lattice_amp=100.0),
]


def _cid(p):
    return f"d{p.dim}-" + "x".join(str(n) for n in p.n) + f"-om{p.omega}"


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("p", CASES, ids=_cid)
def test_apply_h_matches_oracle(dev, p, prec):
    phi = _field(p, 1)
    ref = disc.h_full(p, phi)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    t = torch.from_numpy(phi).to(dt).cuda()
    out, sc = dev.apply_h(p, t, precision=prec)
    got = out.cpu().numpy().astype(np.complex128)
    phi_in = t.cpu().numpy().astype(np.complex128)     # the value the kernel saw
    ref = disc.h_full(p, phi_in)
    tol = _bound(p, phi_in, prec)
    err = float(np.max(np.abs(got - ref)))
    print(f"apply_h {prec} {_cid(p)}: error/bound = {err / tol:.3f}")
    assert err <= tol, (err, tol)
    up = UnifiedProblem(p)
    o = up.outputs(up.to_x(phi_in))
    rtol = 1e-11 if prec == "fp64" else 3e-6
    assert abs(sc["energy"] - o["energy"]) <= rtol * abs(o["energy"])
    assert abs(sc["mu"] - o["mu"]) <= rtol * abs(o["mu"])
    assert abs(sc["norm2"] - up.hvol * float(np.sum(np.abs(phi_in) ** 2))) <= 1e-12
    assert abs(sc["resid"] - o["resid"]) <= tol + rtol * o["resid"]
    for a in range(p.dim):
        assert abs(sc["rms_" + "xyz"[a]] - o["rms"][a]) <= rtol * o["rms"][a] + 1e-14
    assert abs(sc["max_dens"] - o["max_dens"]) <= 1e-12 * o["max_dens"] + 1e-15


def test_apply_h_gaussian_closed_form(dev):
    # beta = 0, Omega = 0 harmonic trap: H phi = (d/2) phi exactly.
    p = W.Problem(dim=2, n=(64, 128), lo=(-12.0, -12.0), hi=(12.0, 12.0))
    x, y = disc.grid_coords(p)
    g = np.exp(-(x * x + y * y) / 2) / math.sqrt(math.pi) + 0j
    out, sc = dev.apply_h(p, torch.from_numpy(g).cuda())
    assert float(np.max(np.abs(out.cpu().numpy() - g))) < 1e-11
    assert abs(sc["energy"] - 1.0) < 1e-12 and sc["resid"] < 1e-11


def test_apply_h_explicit_potential_array(dev):
    p = W.Problem(dim=2, n=(32, 64), lo=(-6.0, -8.0), hi=(6.0, 8.0), beta=50.0, omega=0.5)
    x, y = disc.grid_coords(p)
    v = 0.5 * (x * x + 2 * y * y) + 4.0 * np.exp(-((x - 1) ** 2 + y * y))
    q = W.Problem(dim=2, n=p.n, lo=p.lo, hi=p.hi, beta=p.beta, omega=p.omega, v=v)
    phi = _field(p, 3)
    out, _ = dev.apply_h(p, torch.from_numpy(phi).cuda(), v=torch.from_numpy(v).cuda())
    ref = disc.h_full(q, phi)
    assert float(np.max(np.abs(out.cpu().numpy() - ref))) <= _bound(q, phi, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_h_without_readback(dev, prec):
    # calls without scalars only enqueue work; switching problems between
    # them must still upload each problem's descriptor and V tables
    pa, pb = CASES[6], W.Problem(dim=3, n=(32, 16, 64), lo=(-5.0, -5.0, -9.0), hi=(5.0, 5.0, 9.0),
                                 beta=40.0, omega=-0.2, gamma=(2.0, 1.0, 0.5), lattice_amp=3.0)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    ta = torch.from_numpy(_field(pa, 11)).to(dt).cuda()
    tb = torch.from_numpy(_field(pb, 12)).to(dt).cuda()
    ref_a, _ = dev.apply_h(pa, ta, precision=prec)
    ref_b, _ = dev.apply_h(pb, tb, precision=prec)
    outs = []
    for q, t in ((pa, ta), (pa, ta), (pb, tb), (pa, ta), (pb, tb), (pb, tb)):
        o, sc = dev.apply_h(q, t, precision=prec, scalars=False)
        assert sc is None
        outs.append(o)
    torch.cuda.synchronize()
    for o, ref in zip(outs, (ref_a, ref_a, ref_b, ref_a, ref_b, ref_b)):
        assert torch.equal(o, ref)
    # and the scalars of a later synchronous call are those of its own problem
    _, sa = dev.apply_h(pa, ta, precision=prec)
    o = UnifiedProblem(pa).outputs(UnifiedProblem(pa).to_x(ta.cpu().numpy().astype(np.complex128)))
    assert abs(sa["energy"] - o["energy"]) <= (1e-11 if prec == "fp64" else 3e-6) * abs(o["energy"])


@pytest.mark.parametrize("p", [CASES[1], CASES[3], CASES[6]], ids=_cid)
def test_hess_vec_matches_oracle(dev, p):
    up = UnifiedProblem(p)
    xk = up.to_x(_field(p, 5))
    s = 1e-2 * up.to_x(_field(p, 6))
    delta = 0.37
    ref = up.hess(xk, s) + delta * s
    got = dev.hess_vec(p, torch.from_numpy(xk).cuda(), torch.from_numpy(s).cuda(), delta).cpu().numpy()
    scale = 2 * _bound(p, s / math.sqrt(up.hvol), "fp64") * math.sqrt(up.hvol) \
        + 1e-13 * float(np.max(np.abs(ref)))
    assert float(np.max(np.abs(got - ref))) <= scale


@pytest.mark.parametrize("p", [CASES[1], CASES[3], CASES[5], CASES[6]], ids=_cid)
def test_hess_vec_fp32_matches_oracle(dev, p):
    # mixed precision: s in complex64, transforms in float32, X_k complex128,
    # the pointwise terms in float64 rounded to float32 once on store
    up = UnifiedProblem(p)
    xk = up.to_x(_field(p, 5))
    s32 = (1e-2 * up.to_x(_field(p, 6))).astype(np.complex64)
    s = s32.astype(np.complex128)           # the value the kernel saw
    delta = 0.37
    ref = up.hess(xk, s) + delta * s
    got = dev.hess_vec(p, torch.from_numpy(xk).cuda(), torch.from_numpy(s32).cuda(), delta,
                       precision="mixed").cpu().numpy().astype(np.complex128)
    bound = 2 * _bound(p, s / math.sqrt(up.hvol), "mixed") * math.sqrt(up.hvol) \
        + 2.0 ** -24 * float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(got - ref)))
    print(f"hess_vec fp32 {_cid(p)}: error/bound = {err / bound:.3f}")
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("m", [1, 255, 65536 + 17])
def test_retract_fp32_matches_cayley_closed_form(dev, m):
    # complex64 data, float64 reductions and coefficients
    rng = np.random.default_rng(m + 1)
    x = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex64)
    x /= np.float32(np.linalg.norm(x))
    g = (7.0 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))).astype(np.complex64)
    tau = 0.013
    y, co = dev.retract(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), tau, precision="mixed")
    x64, g64 = x.astype(np.complex128), g.astype(np.complex128)
    a, nx, ng = re_dot(x64, g64), re_dot(x64, x64), re_dot(g64, g64)
    p, q = cayley_coefficients(tau, a, nx, ng)
    assert abs(co["p"] - p) < 1e-12 and abs(co["q"] - q) < 1e-12
    assert abs(co["nx"] - nx) < 1e-12 * nx and abs(co["ng"] - ng) < 1e-12 * ng
    yr = p * x64 + q * g64
    assert y.dtype == torch.complex64
    assert float(np.max(np.abs(y.cpu().numpy().astype(np.complex128) - yr))) <= 2.0 ** -24 * float(np.max(np.abs(yr)))


@pytest.mark.parametrize("m", [1, 255, 65536 + 17])
def test_retract_matches_cayley_closed_form(dev, m):
    rng = np.random.default_rng(m)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    x /= np.linalg.norm(x)
    g = 7.0 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    tau = 0.013
    y, co = dev.retract(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), tau)
    a, nx, ng = re_dot(x, g), re_dot(x, x), re_dot(g, g)
    p, q = cayley_coefficients(tau, a, nx, ng)
    assert abs(co["p"] - p) < 1e-12 and abs(co["q"] - q) < 1e-12
    yr = p * x + q * g
    assert float(np.max(np.abs(y.cpu().numpy() - yr))) < 1e-12 * float(np.max(np.abs(yr)))
    assert abs(np.linalg.norm(y.cpu().numpy()) - 1.0) < 1e-12


@pytest.mark.parametrize("dims", [(32,), (16, 64), (64, 64), (256, 256), (16, 32, 16)])
def test_prolong_matches_oracle(dev, dims):
    d = len(dims)
    pc = W.Problem(dim=d, n=dims, lo=(-5.0,) * d, hi=(7.0,) * d)
    pf = pc.with_n(tuple(2 * n for n in dims))
    rng = np.random.default_rng(2)
    u = rng.standard_normal(pc.shape) + 1j * rng.standard_normal(pc.shape)
    got = dev.prolong(pc, pf, torch.from_numpy(u).cuda()).cpu().numpy()
    ref = prolong_fourier(u)
    n = max(dims)
    assert float(np.max(np.abs(got - ref))) < 1e-13 * n * float(np.max(np.abs(ref)))


# ---------------------------------------------------------------------------
# Sine pseudospectral (Dirichlet, DST-I) operator, §2.2: n intervals, n-1
# interior points per axis.  The oracle's sine path is real (Omega = 0); real
# data go to the GPU as complex with a zero imaginary part.
# ---------------------------------------------------------------------------
SINE_CASES = [
    W.Problem(dim=1, n=(16,), lo=(-4.0,), hi=(4.0,), bc=W.SINE, beta=10.0),
    W.Problem(dim=1, n=(512,), lo=(-16.0,), hi=(16.0,), bc=W.SINE, beta=400.0, lattice_amp=20.0),
    W.Problem(dim=2, n=(32, 64), lo=(-6.0, -8.0), hi=(6.0, 8.0), bc=W.SINE, beta=50.0,
              gamma=(1.0, 1.5, 1.0)),
    W.Problem(dim=2, n=(256, 256), lo=(-16.0, -16.0), hi=(16.0, 16.0), bc=W.SINE, beta=500.0,
              lattice_amp=50.0),
    W.Problem(dim=3, n=(16, 32, 16), lo=(-5.0, -6.0, -4.0), hi=(5.0, 6.0, 4.0), bc=W.SINE, beta=100.0),
    W.Problem(dim=3, n=(128, 128, 128), lo=(-8.0,) * 3, hi=(8.0,) * 3, bc=W.SINE, beta=200.0),
]


def _real_field(p, seed):
    rng = np.random.default_rng(seed)
    cs = disc.grid_coords(p)
    r2 = sum(c * c for c in cs)
    phi = np.exp(-r2 / 4.0) * (1 + 0.3 * cs[0]) + 0.05 * rng.standard_normal(p.shape)
    return phi / math.sqrt(disc.h_vol(p) * float(np.sum(phi * phi)))


def _scid(p):
    return f"sine-d{p.dim}-" + "x".join(str(n) for n in p.n)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("p", SINE_CASES, ids=_scid)
def test_apply_h_sine_matches_oracle(dev, p, prec):
    phi = _real_field(p, 4)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    t = torch.from_numpy(phi.astype(np.complex128)).to(dt).cuda()
    out, sc = dev.apply_h(p, t, precision=prec)
    got = out.cpu().numpy().astype(np.complex128)
    phi_in = t.cpu().numpy().real.astype(np.float64)
    ref = disc.h_full(p, phi_in)
    tol = _bound(p, phi_in, prec)
    assert float(np.max(np.abs(got.real - ref))) <= tol
    assert float(np.max(np.abs(got.imag))) <= tol                # real data stay real
    up = UnifiedProblem(p)
    o = up.outputs(up.to_x(phi_in))
    rtol = 1e-11 if prec == "fp64" else 3e-6
    assert abs(sc["energy"] - o["energy"]) <= rtol * abs(o["energy"])
    assert abs(sc["mu"] - o["mu"]) <= rtol * abs(o["mu"])
    assert abs(sc["norm2"] - up.hvol * float(np.sum(phi_in ** 2))) <= 1e-12
    assert abs(sc["resid"] - o["resid"]) <= tol + rtol * o["resid"]
    for a in range(p.dim):
        assert abs(sc["rms_" + "xyz"[a]] - o["rms"][a]) <= rtol * o["rms"][a] + 1e-14


@pytest.mark.parametrize("p", [SINE_CASES[2], SINE_CASES[4]], ids=_scid)
def test_apply_h_sine_complex_data(dev, p):
    # the kinetic part is linear: kin(a + ib) = kin(a) + i kin(b)
    a, b = _real_field(p, 5), _real_field(p, 6)
    phi = (a + 1j * b) / math.sqrt(2.0)
    out, _ = dev.apply_h(p, torch.from_numpy(phi).cuda())
    kin = disc.kinetic(p, phi.real) + 1j * disc.kinetic(p, phi.imag)
    ref = kin + disc.potential(p) * phi + p.beta * np.abs(phi) ** 2 * phi
    assert float(np.max(np.abs(out.cpu().numpy() - ref))) <= _bound(p, phi, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dims", [(256, 256), (64, 32, 128)])
def test_sine_and_fd_passes_keep_mirror_parity(dev, prec, dims):
    # A field that is exactly odd (or even) under the mirror x -> -x of a
    # centred box gives an H(phi)phi and a Hessian-vector product that are
    # exactly odd (even) too, on lines of every axis (§4.4's excited states
    # are saddle points held by this parity alone).
    d = len(dims)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    for bc in (W.SINE, W.FD):
        p = W.Problem(dim=d, n=dims, lo=(-16.0,) * d, hi=(16.0,) * d, bc=bc, beta=500.0, lattice_amp=50.0)
        f = _real_field(p, 21) + 0.3j * _real_field(p, 22)
        up = UnifiedProblem(p)
        for ax in range(d):
            flip = lambda a: np.flip(a, axis=d - 1 - ax)
            for sgn in (-1.0, 1.0):
                g = 0.5 * (f + sgn * flip(f))
                assert np.array_equal(flip(g), sgn * g)
                t = torch.from_numpy(g).to(dt).cuda()
                out = dev.apply_h(p, t, precision=prec)[0].cpu().numpy()
                assert np.array_equal(flip(out), sgn * out), (bc, ax, sgn, prec)
                xk = math.sqrt(up.hvol) * (np.abs(g) + 0j)     # complex128, even in every axis
                s = dev.hess_vec(p, torch.from_numpy(xk).cuda(), t, 0.37, precision=prec).cpu().numpy()
                assert np.array_equal(flip(s), sgn * s), (bc, ax, sgn, prec, "hess")


def test_apply_h_sine_eigenfunction(dev):
    # beta = 0, V = 0: sin(l pi j / N) x sin(m pi k / N) is an eigenvector of
    # the sine operator with eigenvalue (lambda_l^2 + lambda_m^2) / 2
    p = W.Problem(dim=2, n=(64, 32), lo=(0.0, -1.0), hi=(4.0, 3.0), bc=W.SINE, gamma=(0.0, 0.0, 0.0))
    j = np.arange(1, 64)[None, :]
    k = np.arange(1, 32)[:, None]
    l, m = 5, 3
    f = np.sin(l * np.pi * j / 64) * np.sin(m * np.pi * k / 32) + 0j
    out, _ = dev.apply_h(p, torch.from_numpy(f).cuda())
    lam = 0.5 * ((np.pi * l / 4.0) ** 2 + (np.pi * m / 4.0) ** 2)
    assert float(np.max(np.abs(out.cpu().numpy() - lam * f))) < 1e-12 * lam


def test_apply_h_rotating_3d_eigenfunction(dev):
    # the 3D rotation pin of the oracle on the GPU: eigenvalue 2 - Omega + gz/2
    gz, om = 2.0, 0.4
    p = W.Problem(dim=3, n=(64, 64, 64), lo=(-10.0,) * 3, hi=(10.0,) * 3, omega=om, gamma=(1.0, 1.0, gz))
    x, y, z = disc.grid_coords(p)
    f = (x + 1j * y) * np.exp(-(x * x + y * y) / 2) * np.exp(-gz * z * z / 2)
    out, _ = dev.apply_h(p, torch.from_numpy(np.ascontiguousarray(f)).cuda())
    lam = 2.0 - om + 0.5 * gz
    assert float(np.max(np.abs(out.cpu().numpy() - lam * f))) < 1e-10


# ---------------------------------------------------------------------------
# Second-order finite differences (Dirichlet), §2.1: n intervals, n-1
# interior points per axis, the tridiagonal kinetic matrix per axis.
# ---------------------------------------------------------------------------
FD_CASES = [
    W.Problem(dim=1, n=(16,), lo=(-4.0,), hi=(4.0,), bc=W.FD, beta=10.0),
    W.Problem(dim=1, n=(1024,), lo=(-16.0,), hi=(16.0,), bc=W.FD, beta=400.0, lattice_amp=25.0),
    W.Problem(dim=2, n=(32, 64), lo=(-6.0, -8.0), hi=(6.0, 8.0), bc=W.FD, beta=50.0,
              gamma=(1.0, 1.5, 1.0)),
    W.Problem(dim=2, n=(256, 512), lo=(-16.0, -16.0), hi=(16.0, 16.0), bc=W.FD, beta=500.0,
              lattice_amp=50.0),
    W.Problem(dim=3, n=(16, 32, 64), lo=(-5.0, -6.0, -4.0), hi=(5.0, 6.0, 4.0), bc=W.FD, beta=100.0),
    W.Problem(dim=3, n=(128, 128, 128), lo=(-8.0, -6.0, -4.0), hi=(8.0, 6.0, 4.0), bc=W.FD, beta=200.0,
              gamma=(1.0, 2.0, 4.0)),
]


def _fcid(p):
    return f"fd-d{p.dim}-" + "x".join(str(n) for n in p.n)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("p", FD_CASES, ids=_fcid)
def test_apply_h_fd_matches_oracle(dev, p, prec):
    phi = _real_field(p, 8)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    t = torch.from_numpy(phi.astype(np.complex128)).to(dt).cuda()
    out, sc = dev.apply_h(p, t, precision=prec)
    got = out.cpu().numpy().astype(np.complex128)
    phi_in = t.cpu().numpy().real.astype(np.float64)
    ref = disc.h_full(p, phi_in)
    tol = _bound(p, phi_in, prec)
    assert float(np.max(np.abs(got.real - ref))) <= tol
    assert float(np.max(np.abs(got.imag))) == 0.0                # real data stay exactly real
    up = UnifiedProblem(p)
    o = up.outputs(up.to_x(phi_in))
    rtol = 1e-11 if prec == "fp64" else 3e-6
    assert abs(sc["energy"] - o["energy"]) <= rtol * abs(o["energy"])
    assert abs(sc["mu"] - o["mu"]) <= rtol * abs(o["mu"])
    assert abs(sc["norm2"] - up.hvol * float(np.sum(phi_in ** 2))) <= 1e-12
    assert abs(sc["resid"] - o["resid"]) <= tol + rtol * o["resid"]
    for a in range(p.dim):
        assert abs(sc["rms_" + "xyz"[a]] - o["rms"][a]) <= rtol * o["rms"][a] + 1e-14


def test_apply_h_fd_complex_data(dev):
    p = FD_CASES[4]
    a, b = _real_field(p, 9), _real_field(p, 10)
    phi = (a + 1j * b) / math.sqrt(2.0)
    out, _ = dev.apply_h(p, torch.from_numpy(phi).cuda())
    ref = disc.h_full(p, phi)                       # the FD oracle takes complex data directly
    assert float(np.max(np.abs(out.cpu().numpy() - ref))) <= _bound(p, phi, "fp64")


def test_apply_h_fd_eigenfunction(dev):
    # beta = 0, V = 0: sin(l pi j / N) sin(m pi k / N) is an eigenvector of the
    # tridiagonal kinetic matrices with eigenvalue sum of (2/h^2) sin^2(l pi / 2N)
    p = W.Problem(dim=2, n=(64, 32), lo=(0.0, -1.0), hi=(4.0, 3.0), bc=W.FD, gamma=(0.0, 0.0, 0.0))
    j = np.arange(1, 64)[None, :]
    k = np.arange(1, 32)[:, None]
    l, m = 5, 30
    f = np.sin(l * np.pi * j / 64) * np.sin(m * np.pi * k / 32) + 0j
    out, _ = dev.apply_h(p, torch.from_numpy(f).cuda())
    hx, hy = 4.0 / 64, 4.0 / 32
    lam = 2 / hx ** 2 * math.sin(l * math.pi / 128) ** 2 + 2 / hy ** 2 * math.sin(m * math.pi / 64) ** 2
    assert float(np.max(np.abs(out.cpu().numpy() - lam * f))) < 1e-12 * lam


def test_hess_vec_fd_matches_oracle(dev):
    p = FD_CASES[2]
    up = UnifiedProblem(p)
    # complex X_k and S (the oracle's FD operator is linear over complex data)
    xk = math.sqrt(up.hvol) * (_real_field(p, 11) + 0.2j * _real_field(p, 12))
    s = 1e-2 * math.sqrt(up.hvol) * (_real_field(p, 13) + 0.1j * _real_field(p, 14))
    delta = 0.37
    ref = 2.0 * disc.h_lin(p, s) + 4.0 * up.alpha * (np.abs(xk) ** 2 * s + 2.0 * np.real(np.conj(xk) * s) * xk) \
        + delta * s
    got = dev.hess_vec(p, torch.from_numpy(xk).cuda(), torch.from_numpy(s).cuda(), delta).cpu().numpy()
    scale = 2 * _bound(p, s / math.sqrt(up.hvol), "fp64") * math.sqrt(up.hvol) \
        + 1e-13 * float(np.max(np.abs(ref)))
    assert float(np.max(np.abs(got - ref))) <= scale
