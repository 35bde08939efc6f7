"""Batched launch: many independent instances of uneven size advanced by one
launch per kernel must give, instance by instance, exactly the results of
running each instance alone (same kernels, same per-tile arithmetic), under
every work schedule, and the autotuner must leave the state untouched."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cases():
    out = [synth.acoustic_pulse_case()]
    for n_r, n_t, ustar in ((40, 80, 4.0), (64, 128, 5.0), (50, 96, 6.0)):
        out.append(synth.cylinder_viv_case(n_r=n_r, n_theta=n_t, D=40.0, first_cell_frac=0.025,
                                           r_far_D=10.0, blend_D=4.0, h0_frac=0.01, mstar=2.0,
                                           ustar=ustar))
    return out


def _alone(case, nsteps):
    from paper_2107_01370_amd.fsilbm import Simulation
    s = Simulation(case.mesh, case.fluid, case.bodies)
    s.init_equilibrium(case.rho, case.ux, case.uy, case.T)
    s.step(nsteps)
    f, g = s.populations()
    hist = s.forces(0, nsteps) if case.bodies else None
    state = s.body_state() if case.bodies else None
    s.close()
    return f, g, hist, state


def _batch(cases):
    from paper_2107_01370_amd.fsilbm import Batch
    b = Batch(cases)
    for k, c in enumerate(cases):
        b.init_equilibrium(k, c.rho, c.ux, c.uy, c.T)
    return b


@pytest.fixture(scope="module")
def reference():
    cases = _cases()
    return cases, [_alone(c, 12) for c in cases]


def _compare(b, cases, ref, nsteps, exact=True):
    for k, c in enumerate(cases):
        f, g = b.populations(k)
        if exact:
            assert np.array_equal(f, ref[k][0]) and np.array_equal(g, ref[k][1]), k
        else:
            assert np.max(np.abs(f - ref[k][0])) <= 1e-5 * np.max(np.abs(ref[k][0])), k
            assert np.max(np.abs(g - ref[k][1])) <= 1e-5 * np.max(np.abs(ref[k][1])), k
        if c.bodies and exact:
            assert np.array_equal(b.forces(k, 0, nsteps), ref[k][2]), k
            assert np.array_equal(b.body_state(k), ref[k][3]), k


# the default tile shape of these instances: 32 x 16
DEFAULT = 0


@pytest.mark.parametrize("grid,order,shape", [(0, 0, 0), (0, 1, 0), (16, 0, 0), (64, 1, 0),
                                              (0, 0, 1), (24, 1, 2), (0, 0, 3), (40, 1, 3)])
def test_batch_equals_instances_run_alone(reference, grid, order, shape):
    """Bitwise equal to the instances run alone for their default tile shape;
    the other shapes change only which tile computes a halo node's collision
    (and its FP32 rounding relative to the tile's reference node), so over 12
    steps they agree to 1e-5."""
    cases, ref = reference
    b = _batch(cases)
    b.set_schedule(grid, order, shape)
    b.step(12)
    b.synchronize()
    _compare(b, cases, ref, 12, exact=(shape == DEFAULT))
    b.close()


def test_autotune_keeps_the_state(reference):
    cases, ref = reference
    b = _batch(cases)
    b.step(5)
    grid, order, shape, ms = b.autotune(reps=2)
    assert grid >= 0 and order in (0, 1) and shape in (0, 1, 2, 3) and ms > 0
    b.set_schedule(0, 0, DEFAULT)        # the reference runs used the default shape
    kms = b.time_kernels(2)
    assert kms[0] > 0
    b.step(7)
    b.synchronize()
    _compare(b, cases, ref, 12)
    b.close()


def test_batch_reports_errors_per_instance():
    """An instance driven past one cell per step reports FSI_E_CFL and names itself."""
    from paper_2107_01370_amd.fsilbm import Batch, FsiError
    good = synth.acoustic_pulse_case()
    mesh = synth.cartesian_mesh(64, 16)
    fl = synth.FluidParams(gamma=1.4, Pr=0.71, mu=0.05, T_inf=1 / 3, dt=1.6)
    b = Batch([(good.fluid, good.mesh, []), (fl, mesh, [])])
    b.init_equilibrium(0, good.rho, good.ux, good.uy, good.T)
    b.init_equilibrium(1)
    b.step(1)
    with pytest.raises(FsiError) as e:
        b.synchronize()
    assert e.value.status == -3 and "instance 1" in str(e.value)
    b.close()
