"""Line groups (lb_lines_*): many D1Q3 runs stepped by one kernel launch,
one wavefront per run holding the whole line in registers.

* bit for bit the populations lb_step gives each run alone (every N, line
  length, storage and force form the kernel is built for, parameters that
  differ between the runs of a group, several calls in a row);
* against the FP64 oracle directly;
* a run that becomes unstable is flagged and leaves the others untouched;
* the group's argument checks."""
import numpy as np
import pytest

import lbinputs as LI
from gpu_helpers import TOL, errors, run_oracle

pytestmark = pytest.mark.gpu


def line_cfg(n, L, seed, *, form="log", kappa=0.0):
    """A D1Q3 run with parameters drawn from `seed`: tau, theta, m, chi and
    a noisy sine start."""
    rng = np.random.default_rng(seed)
    m = [float(rng.choice([1.0, 2.0, 10.0])) for _ in range(n)]
    chi = np.zeros((n, n))
    for a in range(n):
        for b in range(a + 1, n):
            # 0.4 to 1.1 times the critical value of the pair alone
            chi_c = 0.5 * (m[a] ** -0.5 + m[b] ** -0.5) ** 2
            chi[a, b] = chi[b, a] = rng.uniform(0.4, 1.1) * chi_c
    p = LI.params("D1Q3", n, (L,), tau=1.0 / rng.uniform(0.7, 1.4), theta=rng.uniform(0.25, 0.45), kappa=kappa,
                  m=m, chi=chi, force_form=form)
    base = np.full(n, 1.0 / n)
    r = LI.noisy_uniform(p, base, 0.1 / n, seed) if n > 1 else LI.noisy_uniform(p, [1.0], 0.1, seed)
    if n > 1:
        r += LI.sine_profile(p, [0.0] * n, amp=0.05)
    return p, r


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_group_equals_lb_step_bitwise(storage, n):
    from paper_0704_3444_amd import Lines, Simulation

    for L in (64, 128, 192, 256):
        runs = [line_cfg(n, L, 100 * n + L + k, form=("log", "expanded")[k % 2], kappa=(0.0, 0.02, 0.05)[k])
                for k in range(3)]
        group_sims = [Simulation(p, r, storage=storage) for p, r in runs]
        alone = [Simulation(p, r, storage=storage) for p, r in runs]
        g = Lines(group_sims)
        for chunk in (1, 37, 100):
            g.step(chunk)
            for s in alone:
                s.step(chunk)
            for k, (a, b) in enumerate(zip(group_sims, alone)):
                fa, fb = a.get_f(), b.get_f()
                assert np.array_equal(fa, fb), (storage, n, L, k, chunk, float(np.abs(fa - fb).max()))
        ma, mb = group_sims[0].moments(), alone[0].moments()
        assert ma["step"] == mb["step"] == 138
        for key in ("rho", "mu", "U", "P", "mass"):
            assert np.array_equal(ma[key], mb[key]), key
        g.close()
        for s in group_sims + alone:
            s.close()
    print(f"[lines] {storage} N={n}: group == lb_step bit for bit, L = 64..256, 138 steps", flush=True)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_group_matches_oracle(storage):
    from paper_0704_3444_amd import Lines, Simulation

    runs = [line_cfg(3, 128, 7), line_cfg(2, 128, 8)]
    for p, r in runs:
        s = Simulation(p, r, storage=storage)
        g = Lines([s])
        g.step(200)
        out = s.moments()
        out["f"] = s.get_f()
        e = errors(out, run_oracle(p, r, 200), p["theta"], lattice=p["lattice"])
        print(f"[lines] {storage} N={p['n_comp']} vs oracle, 200 steps: {e}", flush=True)
        for k in ("rho", "f", "U_cs", "mu", "mom"):
            assert e[k] < TOL[storage], (k, e)
        g.close()
        s.close()


def test_unstable_run_is_flagged_and_isolated():
    """A deep quench without interface energy drives a density to zero and
    the run to NaN; its neighbours in the group are unaffected."""
    from paper_0704_3444_amd import LBError, Lines, Simulation
    from paper_0704_3444_amd.lb import LB_ENUMERIC

    good = [line_cfg(2, 128, 21), line_cfg(2, 128, 22)]
    bad_p = LI.params("D1Q3", 2, (128,), tau=1.0 / 0.9, kappa=0.0, chi=np.array([[0.0, 6.0], [6.0, 0.0]]))
    bad_r = LI.sine_profile(bad_p, [0.5, 0.5], amp=0.1)
    runs = [good[0], (bad_p, bad_r), good[1]]
    sims = [Simulation(p, r) for p, r in runs]
    g = Lines(sims)
    g.step(1000)
    with pytest.raises(LBError) as ei:
        sims[1].moments()
    assert ei.value.code == LB_ENUMERIC
    for k in (0, 2):
        alone = Simulation(*runs[k])
        alone.step(1000)
        assert np.array_equal(alone.get_f(), sims[k].get_f())
        assert sims[k].moments()["status"] == 0
        alone.close()
    g.close()
    for s in sims:
        s.close()


def test_group_argument_checks():
    from paper_0704_3444_amd import LBError, Lines, Simulation
    from paper_0704_3444_amd.lb import LB_EINVAL, LB_ENOTSUP

    a = Simulation(*line_cfg(2, 128, 1))
    b = Simulation(*line_cfg(2, 64, 2))
    c = Simulation(*line_cfg(3, 128, 3))
    cfg2, r2 = LI.binary_spinodal(64)
    d = Simulation(cfg2, r2)
    p5, r5 = line_cfg(2, 320, 4)
    e = Simulation(p5, r5)
    f16 = Simulation(*line_cfg(2, 128, 5), storage="f16s")
    for sims, code in (([a, b], LB_EINVAL), ([a, c], LB_EINVAL), ([a, a], LB_EINVAL), ([d], LB_ENOTSUP),
                       ([e], LB_ENOTSUP), ([f16], LB_ENOTSUP)):
        with pytest.raises(LBError) as ei:
            Lines(sims)
        assert ei.value.code == code
    g = Lines([a])
    a.step(1)  # stepped outside the group: the group refuses to step it
    with pytest.raises(LBError) as ei:
        g.step(1)
    assert ei.value.code == LB_EINVAL
    g.close()
    for s in (a, b, c, d, e, f16):
        s.close()


def test_even_outside_steps_keep_the_group_usable():
    """Two lb_step steps between group calls leave the run on the copy the
    group expects: the group goes on, and the run equals one stepped alone."""
    from paper_0704_3444_amd import Lines, Simulation

    p, r = line_cfg(2, 128, 31)
    a, b = Simulation(p, r), Simulation(*line_cfg(2, 128, 32))
    ref = Simulation(p, r)
    g = Lines([a, b])
    g.step(10)
    a.step(2)
    b.step(2)
    g.step(5)
    ref.step(17)
    assert np.array_equal(a.get_f(), ref.get_f())
    assert a.moments()["step"] == 17
    g.close()
    for s in (a, b, ref):
        s.close()
