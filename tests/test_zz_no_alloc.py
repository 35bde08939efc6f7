"""fsi_step_noalloc, the step for callers that cannot allocate, against
fsi_step through the C ABI.

Both run the same kernels on the same state; the no-allocation step keeps the
step's temporaries (wall masks, targets, tractions, cut staging) in the
library's static device array instead of the workspace and launches directly
instead of replaying a captured graph.  Their populations and load histories
must agree exactly.  Two calls in a row: a C-grid airfoil (wall, cut staging),
then a smaller O-grid cylinder, whose step must not see the first call's
leftovers in the shared array."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def run_both(c, n):
    from paper_2107_01370_amd.fsilbm import Simulation
    ref = Simulation(c.mesh, c.fluid, c.bodies)
    na = Simulation(c.mesh, c.fluid, c.bodies)
    for s in (ref, na):
        s.init_equilibrium(c.rho, c.ux, c.uy, c.T)
    print(f"no-alloc step: {c.mesh.ni}x{c.mesh.nj} topo {c.mesh.topo}, {n} steps", flush=True)
    ref.step(n)
    na.step_noalloc(n)
    na.synchronize()
    fr, gr = ref.populations()
    fa, ga = na.populations()
    hr = ref.forces(0, n + 1)
    ha = na.forces(0, n + 1)
    return (fr, gr, hr), (fa, ga, ha)


def check_equal(ref, na):
    (fr, gr, hr), (fa, ga, ha) = ref, na
    assert np.all(np.isfinite(fa)) and np.all(np.isfinite(ga))
    assert np.array_equal(fa, fr) and np.array_equal(ga, gr)
    assert np.array_equal(ha, hr)


def test_noalloc_step_equals_step_on_two_calls_second_smaller():
    big = synth.small_airfoil_case(alpha0_deg=0.5)
    small = synth.cylinder_viv_case(n_r=32, n_theta=64, D=20.0, first_cell_frac=0.05,
                                    r_far_D=8.0, blend_D=3.0, h0_frac=0.02, mstar=2.0, ustar=4.0)
    assert small.mesh.ni * small.mesh.nj < big.mesh.ni * big.mesh.nj
    r1, a1 = run_both(big, 20)
    check_equal(r1, a1)
    # the loads are not trivial: the airfoil feels a force
    assert np.max(np.abs(a1[2][:, 2])) > 0
    r2, a2 = run_both(small, 20)
    check_equal(r2, a2)
    assert np.max(np.abs(a2[2][:, 2])) > 0


@pytest.mark.parametrize("storage,n_r,n_theta", [(0, 1024, 2048), (1, 2048, 2048)])
def test_noalloc_step_equals_the_split_step(storage, n_r, n_theta):
    """An O-grid whose step streams more than the Infinity Cache (FP32: 1024 x
    2048 nodes; FP16 shifted storage, half the bytes per node: 2048 x 2048),
    on 64 x 8 tiles with non-temporal population stores: fsi_step runs its
    interior tiles on a second stream beside the near-boundary tiles and the
    boundary kernels; the no-allocation step launches every tile at once.
    The two must agree exactly."""
    c = synth.large_heave_case(n_r=n_r, n_theta=n_theta, D=800.0 * n_theta / 2048, storage=storage)
    per_node = 2 * 18 * (4 if storage == 0 else 2) + 16
    assert c.mesh.ni * c.mesh.nj * per_node > 256 << 20
    r, a = run_both(c, 24)
    check_equal(r, a)
    assert np.max(np.abs(a[2][:, 2])) > 0


def test_noalloc_step_refuses_what_it_cannot_hold():
    from paper_2107_01370_amd.fsilbm import FsiError, Simulation
    from synth.unstructured import q9_heave_case
    # 9-node meshes: not supported
    mesh, fl, body, (r, u, v, T) = q9_heave_case()
    sim = Simulation(mesh, fl, [body])
    sim.init_equilibrium(r[None], u[None], v[None], T[None])
    with pytest.raises(FsiError):
        sim.step_noalloc(1)
    # a mesh whose step temporaries exceed the static array (52 B per column)
    wide = synth.cartesian_mesh(32768, 8)
    fluid = synth.FluidParams(gamma=1.4, Pr=0.71, mu=0.01, rho_inf=1.0, T_inf=1.0 / 3.0,
                              u_inf=(0.0, 0.0), dt=1.0 / 3.0)
    sim = Simulation(wide, fluid, [])
    sim.init_equilibrium()
    with pytest.raises(FsiError):
        sim.step_noalloc(1)
    # the ordinary step still runs there
    sim.step(1)
    sim.synchronize()
