"""GPU solver parity against the oracle, through the C ABI.

Protocol (same phi_0 on both sides): (i) relative energy and mu differences,
(ii) the oracle's own residual at the GPU state is below the tolerance,
(iii) ||phi_gpu e^{-i arg<phi_or, phi_gpu>} - phi_or||_inf after phase alignment.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc
from oracle.cascade import cascadic
from oracle.newton import Options, feasible_only, regularized_newton
from oracle.unified import UnifiedProblem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_02891_amd import api
    return api


def _gpu_solve(dev, p, phi0, **opts):
    phi, res = dev.solve(p, torch.from_numpy(np.asarray(phi0, dtype=np.complex128)).cuda(), **opts)
    return phi.cpu().numpy(), res


def _compare(p, phi_gpu, x_or, tol, e_rtol, phi_tol):
    up = UnifiedProblem(p)
    xg = up.to_x(phi_gpu)
    og, oo = up.outputs(xg), up.outputs(x_or)
    assert og["resid"] < tol, og["resid"]                      # (ii)
    assert abs(og["energy"] - oo["energy"]) <= e_rtol * abs(oo["energy"])   # (i)
    assert abs(og["mu"] - oo["mu"]) <= 10 * e_rtol * abs(oo["mu"])
    ph = np.vdot(x_or, xg)
    d = np.max(np.abs(xg * np.conj(ph) / abs(ph) - x_or)) / math.sqrt(up.hvol)
    assert d <= phi_tol, d                                      # (iii)
    return og


def _compare_polished(dev, p, phi_gpu, x_or, tol, e_rtol, polish=1e-10, phi_tol=1e-6):
    """(ii) at the solve's tolerance on the returned state, then (i) and
    (iii) after both sides are polished in FP64 to `polish` (more steps of
    Algorithm 2 from each side's state): a state at residual tol fixes phi
    only to about tol / (spectral gap), the polished states to 1e-6."""
    up = UnifiedProblem(p)
    assert up.outputs(up.to_x(phi_gpu))["resid"] < tol                     # (ii)
    pol, rp = dev.solve(p, torch.from_numpy(np.asarray(phi_gpu, dtype=np.complex128)).cuda(), tol=polish,
                        precision="fp64", max_outer=3000)
    assert rp["status"] == 0, rp
    ref = regularized_newton(up, x_or, Options(tol=polish, max_outer=3000))
    assert ref.converged
    g = pol.cpu().numpy()
    return _compare(p, g if np.iscomplexobj(x_or) else g.real, ref.x, 1.5 * polish, e_rtol, phi_tol)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("beta", [400.0, 0.0])
def test_harmonic_1d_alg2(dev, prec, beta):
    p, phi0 = W.harmonic_1d(beta=beta)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8))
    phi, res = _gpu_solve(dev, p, phi0, tol=1e-8, precision=prec)
    assert res["status"] == 0, res
    assert res["resid"] < 1e-8
    og = _compare(p, phi, ref.x, 1e-8, 1e-10, 1e-6)
    assert abs(og["energy"] - res["energy"]) < 1e-12 * og["energy"]
    if beta == 0.0:
        assert abs(res["energy"] - 0.5) < 1e-12
    # real ground state up to the global phase (a zero mode of the energy);
    # the mixed path keeps its Newton corrections in FP32 (6e-8 relative)
    k = int(np.argmax(np.abs(phi)))
    real = phi * np.conj(phi[k]) / abs(phi[k])
    assert float(np.max(np.abs(real.imag))) < (1e-9 if prec == "fp64" else 1e-6)
    assert abs(res["norm_err"]) < 1e-13


def test_harmonic_1d_alg1_fp64(dev):
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    ref = feasible_only(up, up.to_x(phi0), Options(tol=1e-8))
    phi, res = _gpu_solve(dev, p, phi0, tol=1e-8, algorithm="alg1")
    assert res["status"] == 0
    _compare(p, phi, ref.x, 1e-8, 1e-10, 1e-6)
    # BB trajectories are chaotic at rounding level: perturbing phi_0 by 1e-16
    # relative moves the oracle's own count between 309 and 367 for this
    # problem, so only the order of magnitude is compared
    assert 0.75 * ref.inner <= res["inner_iters"] <= 1.25 * ref.inner, (res["inner_iters"], ref.inner)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rotating_2d_small(dev, prec):
    p = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
    phi0 = W.rotating_initial(p, 0.25, 2)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8, max_outer=3000))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, phi0, tol=1e-8, precision=prec, max_outer=3000)
    assert res["status"] == 0, res
    _compare_polished(dev, p, phi, ref.x, 1e-8, 1e-9)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lattice_3d_small(dev, prec):
    p = W.Problem(dim=3, n=(32, 32, 32), lo=(-8.0,) * 3, hi=(8.0,) * 3, beta=200.0, lattice_amp=25.0)
    phi0 = W.gaussian_times_noise(p, 0.01, 3)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-7))
    phi, res = _gpu_solve(dev, p, phi0, tol=1e-7, precision=prec)
    assert res["status"] == 0, res
    _compare(p, phi, ref.x, 1e-7, 1e-10, 1e-6)


def test_batched_mixed_sizes(dev):
    probs = [W.Problem(dim=2, n=(n, n), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=b, omega=w)
             for n, b, w in ((32, 100.0, 0.0), (64, 300.0, 0.2), (64, 200.0, 0.0))]
    phis = [W.rotating_initial(p, p.omega, 10 + i) for i, p in enumerate(probs)]
    outs, res = dev.solve_batched(probs, [torch.from_numpy(f).cuda() for f in phis], tol=1e-8)
    for p, f, o, r in zip(probs, phis, outs, res):
        up = UnifiedProblem(p)
        ref = regularized_newton(up, up.to_x(f), Options(tol=1e-8))
        assert r["status"] == 0
        _compare_polished(dev, p, o.cpu().numpy(), ref.x, 1e-8, 1e-9)
    # a batched problem follows the same trajectory as when solved alone
    alone, r0 = _gpu_solve(dev, probs[1], phis[1], tol=1e-8)
    assert r0["nfe"] == res[1]["nfe"]
    assert np.array_equal(alone, outs[1].cpu().numpy())


def test_batched_mixed_discretizations(dev):
    # Fourier, sine and finite-difference problems of different sizes in one
    # batch (Omega = 0, real data: real arithmetic for the whole batch); each
    # follows the trajectory it has when solved alone
    mk = lambda n, bc, b: W.Problem(dim=2, n=(n, n), lo=(-8.0, -8.0), hi=(8.0, 8.0), bc=bc, beta=b,
                                    lattice_amp=10.0)
    probs = [mk(32, W.FOURIER, 100.0), mk(64, W.SINE, 300.0), mk(64, W.FD, 200.0), mk(32, W.FD, 50.0)]
    phis = [W.gaussian_times_noise(p, 0.02, 20 + i) + 0j for i, p in enumerate(probs)]
    outs, res = dev.solve_batched(probs, [torch.from_numpy(f).cuda() for f in phis], tol=1e-8,
                                  precision="mixed")
    for i, (p, f, o, r) in enumerate(zip(probs, phis, outs, res)):
        assert r["status"] == 0, (i, r)
        up = UnifiedProblem(p)
        ref = regularized_newton(up, up.to_x(f.real), Options(tol=1e-8))
        _compare_polished(dev, p, o.cpu().numpy().real, ref.x, 1e-8, 1e-9)
        alone, r0 = _gpu_solve(dev, p, f, tol=1e-8, precision="mixed")
        assert r0["nfe"] == r["nfe"], (i, r0["nfe"], r["nfe"])
        assert np.array_equal(alone, o.cpu().numpy()), i


def test_cascadic_two_levels(dev):
    probs = [W.Problem(dim=2, n=(32, 32), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=200.0, omega=w)
             for w in (0.0, 0.3)]
    phis = [W.rotating_initial(p, p.omega, 20 + i) for i, p in enumerate(probs)]
    outs, res = dev.solve_cascadic(probs, [torch.from_numpy(f).cuda() for f in phis], 2,
                                   level_tol=1e-4, tol=1e-8)
    for p, f, o, r in zip(probs, phis, outs, res):
        x_or, pf, _ = cascadic(p, f, (32, 64), Options(tol=1e-8), level_tol=1e-4)
        assert r["status"] == 0
        _compare_polished(dev, pf, o.cpu().numpy(), x_or, 1e-8, 1e-9)


@pytest.mark.parametrize("real", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cascade_equals_its_levels_composed(dev, prec, real):
    # Algorithm 3 as one solve, problems moving between levels on their own,
    # gives each problem the bits of its level-by-level composition: solve to
    # level_tol, prolong, solve the next level, ..., the finest to tol; the
    # evaluation counters add up over the levels.  Real problems (Omega = 0,
    # real data) run every level in the real pair storage.
    if real:
        probs = [W.Problem(dim=2, n=(16, 16), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=b, lattice_amp=a)
                 for b, a in ((200.0, 5.0), (400.0, 0.0), (100.0, 10.0))]
        phis = [W.gaussian_times_noise(p, 0.02, 30 + i) + 0j for i, p in enumerate(probs)]
    else:
        probs = [W.Problem(dim=2, n=(16, 16), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=b, omega=w)
                 for b, w in ((200.0, 0.2), (400.0, 0.6), (100.0, 0.4))]
        phis = [W.rotating_initial(p, p.omega, 30 + i) for i, p in enumerate(probs)]
    levels, ltol, tol = 3, 1e-4, 1e-8
    outs, res = dev.solve_cascadic(probs, [torch.from_numpy(f).cuda() for f in phis], levels,
                                   level_tol=ltol, tol=tol, precision=prec)
    for i, (p, f) in enumerate(zip(probs, phis)):
        cur, pc, nfe, nfe64, inner = torch.from_numpy(f).cuda(), p, 0, 0, 0
        for lv in range(levels):
            # (a prolonged real function carries rounding noise in its imaginary
            # part; the cascade keeps a problem's real storage across levels)
            out, r = dev.solve(pc, cur, tol=ltol if lv < levels - 1 else tol, precision=prec,
                               real_field=1 if real else -1)
            assert r["status"] == 0, (i, lv, r)
            nfe, nfe64, inner = nfe + r["nfe"], nfe64 + r["nfe_fp64"], inner + r["inner_iters"]
            if lv < levels - 1:
                pf = pc.with_n(tuple(2 * n for n in pc.n[:pc.dim]))
                cur, pc = dev.prolong(pc, pf, out), pf
        assert res[i]["status"] == 0, (i, res[i])
        assert res[i]["storage"] == (2 if real else 0), res[i]
        assert (res[i]["nfe"], res[i]["nfe_fp64"], res[i]["inner_iters"]) == (nfe, nfe64, inner), i
        assert np.array_equal(out.cpu().numpy(), outs[i].cpu().numpy()), i


def test_error_paths(dev):
    from paper_1504_02891_amd.api import GpeError
    p, phi0 = W.harmonic_1d(beta=10.0)
    z = torch.zeros(512, dtype=torch.complex128, device="cuda")
    with pytest.raises(GpeError) as e:
        dev.solve(p, z)
    assert e.value.status == -1                                 # zero phi_0
    bad = phi0.astype(np.complex128).copy()
    bad[7] = np.nan
    with pytest.raises(GpeError) as e:
        dev.solve(p, torch.from_numpy(bad).cuda())
    assert e.value.status == -5
    q = W.Problem(dim=1, n=(48,), lo=(-4.0,), hi=(4.0,))
    with pytest.raises(GpeError) as e:
        dev.apply_h(q, torch.zeros(48, dtype=torch.complex128, device="cuda"))
    assert e.value.status == -2
    r = W.Problem(dim=1, n=(64,), lo=(-4.0,), hi=(4.0,), omega=0.5)
    with pytest.raises(GpeError) as e:
        dev.apply_h(r, torch.zeros(64, dtype=torch.complex128, device="cuda"))
    assert e.value.status == -1
    phi, res = dev.solve(p, torch.from_numpy(phi0 + 0j).cuda(), max_outer=0, k_init=1, tol=1e-14)
    assert res["status"] == 1 and np.isfinite(res["energy"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_and_plain_launches_agree(dev, prec):
    # the host loop launches each chunk ahead of the check of the one before,
    # as a replayed hipGraph or as plain launches (profiling forces plain
    # launches and checks in turn): the same evaluations, the same bits
    p = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
    phi0 = W.rotating_initial(p, 0.25, 2)
    outs = []
    for kw in (dict(use_graph=1), dict(use_graph=0), dict(use_graph=0, profile=7)):
        phi, res = _gpu_solve(dev, p, phi0, tol=1e-8, precision=prec, **kw)
        assert res["status"] == 0, (kw, res)
        outs.append((phi, res["nfe"], res["energy"]))
    for phi, nfe, e in outs[1:]:
        assert nfe == outs[0][1] and e == outs[0][2]
        assert np.array_equal(phi, outs[0][0])


def test_cascade_error_paths(dev):
    # a level past 1024 points per axis, a sine problem, and a problem whose
    # data are not finite: its coarse level ends in error and the cascade
    # still hands back a finest-grid array (its coarse iterate prolonged)
    from paper_1504_02891_amd.api import GpeError
    p = W.Problem(dim=2, n=(512, 512), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=100.0, omega=0.2)
    f = torch.from_numpy(W.rotating_initial(p, 0.2, 3)).cuda()
    with pytest.raises(GpeError) as e:
        dev.solve_cascadic([p], [f], 3)          # 512 -> 1024 -> 2048
    assert e.value.status == -2
    q = W.Problem(dim=2, n=(32, 32), lo=(-8.0, -8.0), hi=(8.0, 8.0), bc=W.SINE, beta=100.0)
    with pytest.raises(GpeError) as e:
        dev.solve_cascadic([q], [torch.ones((31, 31), dtype=torch.complex128, device="cuda")], 2)
    assert e.value.status == -2
    r = W.Problem(dim=2, n=(32, 32), lo=(-8.0, -8.0), hi=(8.0, 8.0), beta=100.0, omega=0.3)
    g = W.rotating_initial(r, 0.3, 4)
    g[5, 7] = np.nan
    with pytest.raises(GpeError) as e:
        dev.solve_cascadic([r], [torch.from_numpy(g).cuda()], 3)
    assert e.value.status == -5


@pytest.mark.parametrize("case", ["rot2d-mixed", "lattice3d-fp64", "lattice3d-128-mixed-capped"])
def test_step_placements_agree(dev, case):
    # where the scalar step runs (own launch, last workgroup of the final
    # pass) and how the evaluations are grouped (graph chunk length; plain
    # launches) must not change a single bit of the result.  At 128^3 with
    # 128-thread tiles (2048 final tiles) the step kernel spreads its
    # reductions over its wavefronts slot by slot while the last workgroup
    # (two wavefronts) reduces every slot in one: the same bits either way
    tol, max_outer, ok, extra = 1e-8, 3000, 0, {}
    if case == "rot2d-mixed":
        p = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
        phi0, prec = W.rotating_initial(p, 0.25, 2), "mixed"
    elif case == "lattice3d-fp64":
        p = W.Problem(dim=3, n=(32, 32, 32), lo=(-8.0,) * 3, hi=(8.0,) * 3, beta=200.0, lattice_amp=25.0)
        phi0, prec = W.gaussian_times_noise(p, 0.01, 3), "fp64"
    else:
        p, phi0 = W.lattice_3d()
        prec, tol, max_outer, ok, extra = "mixed", 1e-12, 2, 1, dict(threads=[128, 128, 128])
    runs = [dict(step_at="kernel"), dict(step_at="last_group"), dict(step_at="auto"),
            dict(step_at="last_group", chunk=7), dict(step_at="kernel", chunk=7),
            dict(step_at="last_group", use_graph=0, chunk=16), dict(step_at="fused"),
            dict(step_at="fused", chunk=7), dict(step_at="fused", use_graph=0, chunk=16)]
    out = [_gpu_solve(dev, p, phi0, tol=tol, precision=prec, max_outer=max_outer, **extra, **kw) for kw in runs]
    phi_ref, r_ref = out[0]
    assert r_ref["status"] == ok, r_ref
    for (phi, r), kw in zip(out[1:], runs[1:]):
        assert r["status"] == r_ref["status"], kw
        for k in ("nfe", "nfe_fp64", "outer_iters", "inner_iters", "backtracks", "rejections"):
            assert r[k] == r_ref[k], (kw, k, r[k], r_ref[k])
        assert np.array_equal(phi, phi_ref), kw



@pytest.mark.parametrize("case", ["sine-1d", "sine-2d-lattice", "sine-3d"])
def test_sine_ground_state(dev, case):
    # Dirichlet (sine pseudospectral) ground states, real initial data; the
    # oracle runs the same algorithm in real arithmetic
    if case == "sine-1d":
        p = W.Problem(dim=1, n=(128,), lo=(-16.0,), hi=(16.0,), bc=W.SINE, beta=400.0)
        phi0, tol = W.gaussian_times_noise(p, 0.05, 1), 1e-8
    elif case == "sine-2d-lattice":
        p = W.Problem(dim=2, n=(64, 64), lo=(-16.0, -16.0), hi=(16.0, 16.0), bc=W.SINE, beta=500.0,
                      lattice_amp=50.0)
        phi0, tol = W.gaussian_times_noise(p, 0.01, 7), 1e-8
    else:
        p = W.Problem(dim=3, n=(32, 32, 32), lo=(-8.0,) * 3, hi=(8.0,) * 3, bc=W.SINE, beta=200.0,
                      lattice_amp=25.0)
        phi0, tol = W.gaussian_times_noise(p, 0.01, 3), 1e-7
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=tol))
    assert ref.converged
    for prec in ("fp64", "mixed"):
        # real phi_0 and Omega = 0: real arithmetic is chosen automatically
        phi, res = _gpu_solve(dev, p, phi0.astype(np.complex128), tol=tol, precision=prec)
        assert res["status"] == 0, (prec, res)
        assert np.all(phi.imag == 0.0), prec
        _compare(p, phi.real, ref.x, tol, 1e-10, 1e-6)


@pytest.mark.parametrize("case", ["fd-1d", "fd-2d-lattice", "fd-3d"])
def test_fd_ground_state(dev, case):
    # finite-difference (Dirichlet) ground states against the oracle's
    # tridiagonal operator, both precisions, real initial data
    if case == "fd-1d":
        p = W.Problem(dim=1, n=(128,), lo=(-16.0,), hi=(16.0,), bc=W.FD, beta=400.0)
        phi0, tol = W.gaussian_times_noise(p, 0.05, 1), 1e-8
    elif case == "fd-2d-lattice":
        p = W.Problem(dim=2, n=(64, 64), lo=(-16.0, -16.0), hi=(16.0, 16.0), bc=W.FD, beta=500.0,
                      lattice_amp=50.0)
        phi0, tol = W.gaussian_times_noise(p, 0.01, 7), 1e-8
    else:
        p = W.Problem(dim=3, n=(32, 32, 32), lo=(-8.0, -6.0, -4.0), hi=(8.0, 6.0, 4.0), bc=W.FD,
                      beta=200.0, gamma=(1.0, 2.0, 4.0))
        phi0, tol = W.gaussian_times_noise(p, 0.01, 3), 1e-7
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=tol))
    assert ref.converged
    for prec in ("fp64", "mixed"):
        phi, res = _gpu_solve(dev, p, phi0.astype(np.complex128), tol=tol, precision=prec)
        assert res["status"] == 0, (prec, res)
        assert np.all(phi.imag == 0.0), prec
        if tol < 1e-7:
            _compare(p, phi.real, ref.x, tol, 1e-10, 1e-6)
        else:
            _compare_polished(dev, p, phi.real, ref.x, tol, 1e-10)


def test_fd_accuracy_row_sec4_1(dev):
    # §4.1 Case I at h = 1/4 (128 intervals on (-16, 16)): the GPU's
    # finite-difference ground state reproduces the printed |E_g - E_h| and
    # |mu_g - mu_h|, with E_g, mu_g from the GPU's sine solve at h = 1/16
    from conftest import read_golden
    gold = read_golden("fd_accuracy_1d.txt")
    k = gold["h"].index(0.25)
    ps = W.Problem(dim=1, n=(512,), lo=(-16.0,), hi=(16.0,), bc=W.SINE, beta=400.0)
    pf = W.Problem(dim=1, n=(128,), lo=(-16.0,), hi=(16.0,), bc=W.FD, beta=400.0)
    g = lambda p: np.exp(-disc.grid_coords(p)[0] ** 2 / 8) + 0j
    _, rs = _gpu_solve(dev, ps, g(ps), tol=1e-11, algorithm="alg1")
    _, rf = _gpu_solve(dev, pf, g(pf), tol=1e-11, algorithm="alg1")
    assert rs["status"] == 0 and rf["status"] == 0
    for key in ("energy", "mu"):
        ref = gold[f"case1_{key}"][k]
        assert abs(abs(rs[key] - rf[key]) - ref) <= 0.01 * ref, (key, rs[key], rf[key], ref)


def test_sine_rejections(dev):
    from paper_1504_02891_amd.api import GpeError
    p = W.Problem(dim=2, n=(32, 32), lo=(-4.0, -4.0), hi=(4.0, 4.0), bc=W.SINE, omega=0.3)
    z = torch.ones(31 * 31, dtype=torch.complex128, device="cuda")
    with pytest.raises(GpeError) as e:
        dev.solve(p, z)                                            # rotation needs Fourier
    assert e.value.status == -1
    q = W.Problem(dim=1, n=(1024,), lo=(-4.0,), hi=(4.0,), bc=W.SINE)
    with pytest.raises(GpeError) as e:
        dev.apply_h(q, torch.ones(1023, dtype=torch.complex128, device="cuda"))
    assert e.value.status == -2                                    # 2n-point extension > 1024
    with pytest.raises(ValueError):
        dev.apply_h(W.Problem(dim=1, n=(64,), lo=(-4.0,), hi=(4.0,), bc=W.SINE),
                    torch.ones(64, dtype=torch.complex128, device="cuda"))   # needs 63 values



def test_real_field_option(dev):
    from paper_1504_02891_amd.api import GpeError
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8))
    # complex phi_0 (a global phase) with Omega = 0: complex arithmetic; the
    # result is the ground state times a phase
    phi, res = _gpu_solve(dev, p, phi0 * np.exp(0.3j), tol=1e-8)
    assert res["status"] == 0
    assert float(np.max(np.abs(phi.imag))) > 1e-3
    _compare(p, phi, ref.x, 1e-8, 1e-10, 1e-6)
    # forced real arithmetic drops the phase's imaginary part at the start
    phi, res = _gpu_solve(dev, p, phi0 + 0j, tol=1e-8, real_field=1, precision="mixed")
    assert res["status"] == 0 and np.all(phi.imag == 0.0)
    _compare(p, phi.real, ref.x, 1e-8, 1e-10, 1e-6)
    # complex arithmetic on real data still works (rounding may rotate the phase)
    phi, res = _gpu_solve(dev, p, phi0 + 0j, tol=1e-8, real_field=0)
    assert res["status"] == 0
    _compare(p, phi, ref.x, 1e-8, 1e-10, 1e-6)
    # real arithmetic needs Omega = 0
    q = W.Problem(dim=2, n=(32, 32), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=100.0, omega=0.2)
    with pytest.raises(GpeError) as e:
        dev.solve(q, torch.from_numpy(W.rotating_initial(q, 0.2, 1)).cuda(), real_field=1)
    assert e.value.status == -1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["2d-explicit-v", "3d-lattice"])
def test_real_pair_storage(dev, case, prec):
    # real data on a Fourier grid at Omega = 0: the solver keeps real values,
    # two grid points to a complex element (storage 2), and reaches the
    # oracle's ground state as the complex storage (real_field = 0) does; the
    # 2D case reads an explicit, x-asymmetric potential array in pair storage
    if case == "2d-explicit-v":
        q = W.Problem(dim=2, n=(64, 32), lo=(-8.0, -6.0), hi=(8.0, 6.0), beta=300.0)
        x, y = disc.grid_coords(q)
        v = 0.5 * (x * x + 2.0 * y * y) + 0.3 * x + 2.0 * np.sin(np.pi * x / 4) ** 2
        p = W.Problem(dim=2, n=(64, 32), lo=(-8.0, -6.0), hi=(8.0, 6.0), beta=300.0, v=v)
        phi0 = W.gaussian_times_noise(p, 0.02, 41)
        vt = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    else:
        p = W.Problem(dim=3, n=(32, 32, 16), lo=(-8.0,) * 3, hi=(8.0,) * 3, beta=200.0, lattice_amp=10.0)
        phi0, vt = W.gaussian_times_noise(p, 0.02, 42), None
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8))
    assert ref.converged
    for rf, storage in ((-1, 2), (0, 0)):
        out, res = dev.solve(p, torch.from_numpy(np.asarray(phi0 + 0j, dtype=np.complex128)).cuda(), v=vt,
                             tol=1e-8, precision=prec, real_field=rf)
        assert res["status"] == 0 and res["storage"] == storage, res
        phi = out.cpu().numpy()
        if storage == 2:
            assert np.all(phi.imag == 0.0)
            _compare(p, phi.real, ref.x, 1e-8, 1e-10, 1e-6)
        else:
            _compare(p, phi, ref.x, 1e-8, 1e-10, 1e-6)


def test_stop_rule_crit1_sine_1d(dev):
    # §4.1: Algorithm 1 on the sine discretization, crit1 with eps0 = 1e-12,
    # reproduces the printed values; the oracle runs the same rule
    gold = {"energy": 21.3601, "mu": 35.5775, "x_rms": 3.7751}
    p = W.Problem(dim=1, n=(256,), lo=(-16.0,), hi=(16.0,), bc=W.SINE, beta=400.0)
    xs = disc.axis_points(p, 0)
    f0 = np.exp(-xs * xs / 2) + 0j
    up = UnifiedProblem(p)
    ref = feasible_only(up, up.to_x(f0.real), Options(stop_rule="crit1", eps0=1e-12))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, f0, algorithm="alg1", stop_rule="crit1", eps0=1e-12, tol=0.0)
    assert res["status"] == 0, res
    assert round(res["energy"], 4) == gold["energy"] and round(res["mu"], 4) == gold["mu"]
    assert round(res["rms"][0], 4) == gold["x_rms"]
    _compare(p, phi.real, ref.x, 1e-9, 1e-12, 1e-8)
    assert abs(res["inner_iters"] - ref.inner) <= 0.25 * ref.inner, (res["inner_iters"], ref.inner)
    # eps0 = inf: the first accepted step stops Algorithm 1
    for prec in ("fp64", "mixed"):
        _, r1 = _gpu_solve(dev, p, f0, algorithm="alg1", stop_rule="crit1", eps0=math.inf, precision=prec)
        assert r1["status"] == 0 and r1["inner_iters"] == 1, (prec, r1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_stop_rule_crit2_newton(dev, prec):
    # Algorithm 2 stopped by crit2 on accepted Newton steps
    p = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
    phi0 = W.rotating_initial(p, 0.25, 2)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(stop_rule="crit2", crit2_tol=1e-8))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, phi0, stop_rule="crit2", crit2_tol=1e-8, precision=prec)
    assert res["status"] == 0, res
    # the step rule bounds the step, not the residual: compare energies, and
    # the state loosely (the oracle's residual at its own stop is the scale)
    og = up.outputs(ref.x)
    assert abs(res["energy"] - og["energy"]) <= 1e-9 * og["energy"]
    assert res["resid"] < 100 * max(og["resid"], 1e-7)
    # crit2_tol = inf: the evaluation after the first accepted Newton step stops
    _, r2 = _gpu_solve(dev, p, phi0, stop_rule="crit2", crit2_tol=math.inf, precision=prec)
    assert r2["status"] == 0 and r2["outer_iters"] == r2["rejections"] + 1, r2


def test_monotone_search(dev):
    # monotone Armijo (eta = 0) on the GPU follows the oracle's monotone run
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    ref = feasible_only(up, up.to_x(phi0), Options(tol=1e-8, monotone=True))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, phi0 + 0j, algorithm="alg1", monotone=1, tol=1e-8)
    assert res["status"] == 0, res
    _compare(p, phi.real, ref.x, 1e-8, 1e-10, 1e-6)
    assert abs(res["inner_iters"] - ref.inner) <= 0.25 * ref.inner, (res["inner_iters"], ref.inner)


_LATTICE_XFAIL = pytest.mark.xfail(
    reason="the A = 50 lattice wells are weakly coupled, so stationary states whose lobes differ in "
           "sign lie within 1e-4 of the ground state; which one Algorithm 1's BB iteration reaches "
           "depends on FP32 rounding (one build's run ended in the state with the central lobe "
           "flipped, E 3.2e-5 above the ground state, r = 7e-7)", strict=False)


def _mirror_part(f, odd_x, odd_y):
    """The part of f with the given parity under the mirrors x -> -x, y -> -y
    of a centred box (array axes: y, x), exactly (a + b and a - b are exact
    negatives or equals at mirror points)."""
    g = 0.5 * (f - f[:, ::-1]) if odd_x else 0.5 * (f + f[:, ::-1])
    return 0.5 * (g - g[::-1, :]) if odd_y else 0.5 * (g + g[::-1, :])


_EXCITED_FP32_XFAIL = pytest.mark.xfail(
    reason="within a parity class the A = 50 lattice has several stationary states (its wells are "
           "weakly coupled); FP32 rounding in the early steps of Algorithm 1 can lead to another one "
           "of the same parity (one run reached E = 34.6500 instead of phi_10's 34.6053, exactly odd, "
           "r < 1e-6 after the FP64 continuation); FP64 reproduces Table 10", strict=False)


@pytest.mark.parametrize("key,prec", [
    ("phi_g", "fp64"), pytest.param("phi_g", "mixed", marks=_LATTICE_XFAIL),
    ("phi_10", "fp64"), pytest.param("phi_10", "mixed", marks=_EXCITED_FP32_XFAIL),
    ("phi_11", "fp64"), pytest.param("phi_11", "mixed", marks=_EXCITED_FP32_XFAIL)])
def test_excited_states_sine_2d(dev, key, prec):
    # §4.4 (Table 10): Algorithm 1 on the sine discretization, 255^2 interior
    # points, beta = 500, lattice A = 50; initial data of a mirror parity stay
    # in their parity class (the sine passes keep an exactly odd or even line
    # exactly so) and reach the excited states.  Printed to four decimals.
    # Mixed precision reaches tol = 1e-6 through the FP64 continuation.
    from conftest import read_golden
    gold = read_golden("table10_sp2d.txt")
    p = W.Problem(dim=2, n=(256, 256), lo=(-16.0, -16.0), hi=(16.0, 16.0), bc=W.SINE, beta=500.0,
                  lattice_amp=50.0)
    x, y = disc.grid_coords(p)
    e = np.exp(-(x * x + y * y) / 2) / math.sqrt(math.pi)
    f = {"phi_g": e + 0 * x, "phi_10": math.sqrt(2) * x * e, "phi_11": 2 * x * y * e}[key]
    odd = {"phi_g": (False, False), "phi_10": (True, False), "phi_11": (True, True)}[key]
    f = _mirror_part(f, *odd)
    phi, res = _gpu_solve(dev, p, f + 0j, algorithm="alg1", tol=1e-6, precision=prec)
    assert res["status"] == 0, (key, res)
    # the result keeps the parity of the initial data exactly
    assert np.array_equal(phi, _mirror_part(phi, *odd)), key
    got = [res["max_dens"], res["energy"], res["mu"], res["rms"][0], res["rms"][1]]
    assert [round(v, 4) for v in got] == gold[key], (key, got)


def test_mixed_alg1_switches_to_fp64(dev):
    # below the FP32 floor, mixed-precision Algorithm 1 continues in FP64
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    ref = feasible_only(up, up.to_x(phi0), Options(tol=1e-10))
    phi, res = _gpu_solve(dev, p, phi0 + 0j, algorithm="alg1", tol=1e-10, precision="mixed")
    assert res["status"] == 0 and res["resid"] < 1e-10, res
    assert 0 < res["switch_iter"] < res["inner_iters"], res
    assert res["nfe_fp64"] > 0
    _compare(p, phi.real, ref.x, 1e-10, 1e-12, 1e-8)
    # switch_window = 0: no switch; the FP32 run ends at the step cap
    _, r0 = _gpu_solve(dev, p, phi0 + 0j, algorithm="alg1", tol=1e-10, precision="mixed",
                       switch_window=0, max_iter=3000)
    assert r0["status"] == 1 and r0["switch_iter"] == 0


@pytest.mark.parametrize("case", ["lattice-3d", "rotating-2d"])
def test_mixed_alg2_hands_over_to_fp64(dev, case):
    # mixed Algorithm 2 hands X_k to an FP64 run of Algorithm 2 once an outer
    # residual is below switch_resid; with switch_resid = 0 it stays mixed
    if case == "lattice-3d":
        p = W.Problem(dim=3, n=(32, 32, 32), lo=(-8.0,) * 3, hi=(8.0,) * 3, beta=200.0, lattice_amp=25.0)
        phi0, tol, sw = W.gaussian_times_noise(p, 0.01, 3), 1e-7, 1e-4
    else:
        p = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
        phi0, tol, sw = W.rotating_initial(p, 0.25, 2), 1e-8, 1e-5
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=tol, max_outer=3000))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, phi0, tol=tol, precision="mixed", switch_resid=sw, max_outer=3000)
    assert res["status"] == 0 and res["resid"] < tol, res
    assert 0 < res["switch_iter"] <= res["inner_iters"], res
    assert res["nfe_fp64"] > res["nfe_outer"], res        # FP64 Algorithm 1 steps after the handover
    # evaluation accounting: every evaluation has one mode; the mixed passes ran
    # part of them, the FP64 continuation the rest
    assert res["nfe_f"] + res["nfe_w"] + res["nfe_outer"] == res["nfe"], res
    assert all(0 <= a <= b for a, b in zip(res["nfe_mixed"], (res["nfe_f"], res["nfe_w"], res["nfe_outer"]))), res
    assert res["nfe_mixed"][0] > 0 and res["nfe_mixed"][2] > 0, res   # K_init steps; the handover's outer evaluation
    assert sum(res["nfe_mixed"]) < res["nfe"], res
    _compare_polished(dev, p, phi, ref.x, tol, 1e-9)
    phi0_, r0 = _gpu_solve(dev, p, phi0, tol=tol, precision="mixed", switch_resid=0.0, max_outer=3000)
    assert r0["status"] == 0 and r0["switch_iter"] == 0, r0
    assert r0["nfe_mixed"] == [r0["nfe_f"], r0["nfe_w"], r0["nfe_outer"]], r0
    _compare_polished(dev, p, phi0_, ref.x, tol, 1e-9)
    _, r64 = _gpu_solve(dev, p, phi0, tol=tol, precision="fp64", max_outer=3000)
    assert r64["nfe_mixed"] == [0, 0, 0] and r64["switch_iter"] == 0, r64


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rotating_3d_small(dev, prec):
    # 3D rotating Fourier problem (rotation about z), Algorithm 2 vs the oracle
    p = W.Problem(dim=3, n=(32, 32, 32), lo=(-7.0,) * 3, hi=(7.0,) * 3, beta=300.0, omega=0.5,
                  gamma=(1.0, 1.0, 1.5))
    phi0 = W.rotating_initial(p, 0.5, 9) * np.exp(-0.75 * disc.grid_coords(p)[2] ** 2)
    up = UnifiedProblem(p)
    ref = regularized_newton(up, up.to_x(phi0), Options(tol=1e-7, max_outer=3000))
    assert ref.converged
    phi, res = _gpu_solve(dev, p, phi0, tol=1e-7, precision=prec, max_outer=3000)
    assert res["status"] == 0, res
    _compare_polished(dev, p, phi, ref.x, 1e-7, 1e-9, polish=1e-8)   # (the oracle's polish to 1e-9 takes minutes)


def test_set_plan(dev):
    # a plan given to the context is used by later solves with open launch
    # options: bitwise the same as passing it explicitly (a grid no other test
    # uses, since the plan stays in the context); invalid plans are refused
    from paper_1504_02891_amd.api import GpeError
    p = W.Problem(dim=2, n=(128, 32), lo=(-10.0, -6.0), hi=(10.0, 6.0), beta=300.0, omega=0.2)
    phi0 = W.rotating_initial(p, 0.2, 13)
    for ept in ([8, 8, 0], [4, 4, 0]):
        dev.set_plan(p, "fp64", [64, 64, 0], 1, elems=ept)
        phi_a, ra = _gpu_solve(dev, p, phi0, tol=1e-8, precision="fp64")
        phi_b, rb = _gpu_solve(dev, p, phi0, tol=1e-8, precision="fp64", threads=[64, 64, 0], elems=ept,
                               step_at="kernel")
        assert ra["status"] == 0 and ra["nfe"] == rb["nfe"]
        assert np.array_equal(phi_a, phi_b)
    for thr, sa, ept in (([32, 64, 0], 1, None), ([64, 96, 0], 1, None), ([64, 64, 0], 5, None),
                         ([64, 64, 0], 3, None), ([64, 64, 0], 1, [5, 8, 8]), ([64, 64, 0], 1, [8, 2, 8])):
        with pytest.raises(GpeError) as e:
            dev.set_plan(p, "fp64", thr, sa, elems=ept)
        assert e.value.status == -1


def test_autotune_plan(dev):
    # the tuned plan is a valid configuration, and a later solve with open
    # launch options uses it: bitwise the same as the plan given explicitly
    # (a grid no other test uses, since the plan stays in the context)
    p = W.Problem(dim=2, n=(128, 64), lo=(-10.0, -8.0), hi=(10.0, 8.0), beta=400.0, omega=0.3)
    plan = dev.autotune(p, "mixed")
    assert plan["us_per_eval"] > 0.0 and plan["step_at"] in (0, 1, 2)
    for a, n in enumerate(p.n):
        t, e = plan["threads"][a], plan["elems"][a]
        assert e in (4, 8) and t in (64, 128, 256) and t % (n // e) == 0, plan
    phi0 = W.rotating_initial(p, 0.3, 12)
    # no FP64 continuation: its passes would take the FP64 plan of the grid
    # in one run and the given threads in the other
    phi_a, ra = _gpu_solve(dev, p, phi0, tol=1e-8, precision="mixed", switch_resid=0.0)
    phi_b, rb = _gpu_solve(dev, p, phi0, tol=1e-8, precision="mixed", threads=plan["threads"][:2] + [0],
                           elems=plan["elems"][:2] + [0], step_at=plan["step_at"], switch_resid=0.0)
    assert ra["status"] == 0 and ra["nfe"] == rb["nfe"]
    assert np.array_equal(phi_a, phi_b)
