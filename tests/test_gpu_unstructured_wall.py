"""GPU parity on an unstructured 9-node mesh round a cylinder, fixed or moving
(missing populations where departure points leave the mesh, free-stream far
field, Grad wall populations with targets at B and nodal finite-element
gradients, force over the wall polygon; blended mesh motion with the
departure points relocated every step) against the FP64 oracle, through the
C ABI."""

from dataclasses import replace

import numpy as np
import pytest

from oracle.unstructured import UnstructuredWallSolver
from synth.unstructured import q9_cylinder_case

pytestmark = pytest.mark.gpu


def paired(case, storage=0):
    from paper_2107_01370_amd.fsilbm import Simulation
    mesh, fl, body, (rho, ux, uy, T) = case
    sim = Simulation(mesh, replace(fl, storage=storage), [body])
    sim.init_equilibrium(rho[None], ux[None], uy[None], T[None])
    f0, g0 = sim.populations()
    ora = UnstructuredWallSolver(mesh, fl, body, rho, ux, uy, T)
    if storage == 0:
        ora.f = f0[:, 0, :].astype(np.float64)
        ora.g = g0[:, 0, :].astype(np.float64)
    return sim, ora


def test_wall_one_step_population_parity():
    sim, ora = paired(q9_cylinder_case())
    sim.step(1)
    ora.step()
    f, g = sim.populations()
    for a, b in ((f[:, 0, :], ora.f), (g[:, 0, :], ora.g)):
        err = np.abs(a - b)
        assert np.max(err) <= 1e-6 * np.max(np.abs(b)), (np.unravel_index(np.argmax(err), err.shape),
                                                         np.max(err))


def test_wall_60_steps_fields_and_forces():
    sim, ora = paired(q9_cylinder_case(seed=3))
    n = 60
    sim.step(n)
    ora.run(n)
    rho, ux, uy, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    assert np.array_equal(hist[:, 0], ho[:, 0])
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert fscale > 0
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale


def test_wall_mirror_mesh_keeps_lift_at_rounding_level():
    sim, ora = paired(q9_cylinder_case(mirror=True))
    sim.step(80)
    h = sim.forces(0, 81)
    assert h[-1, 1] > 0.1
    assert np.max(np.abs(h[:, 2])) <= 1e-4 * h[-1, 1]


def test_wall_fp16_storage_within_2e3():
    """FP16 shifted storage rounds every population every step; with this
    mesh's small time step (dt = 0.05, the near-wall elements are a quarter
    of a lattice unit) the rounding accumulates over 6-7 times more steps per
    unit time than on the structured meshes (2.3e-3 after 40 steps, growing
    steadily from 2e-4 after one), so the bar is taken after 20 steps."""
    case = q9_cylinder_case(seed=4)
    sim, ora = paired(case, storage=1)
    sim.step(20)
    ora.run(20)
    r, _, _, Tg = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(r[0] - r_o) / r_o) <= 2e-3
    assert np.max(np.abs(r[0] * Tg[0] - r_o * T_o) / (r_o * T_o)) <= 2e-3


def test_wall_checkpoint_and_single_steps_keep_the_run():
    from paper_2107_01370_amd.fsilbm import Simulation
    mesh, fl, body, (rho, ux, uy, T) = q9_cylinder_case(seed=5)

    def fresh():
        s = Simulation(mesh, fl, [body])
        s.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        return s

    a = fresh()
    a.step(7)
    ckpt = a.save()
    a.step(20)
    b = fresh()
    b.load(ckpt)
    for _ in range(20):
        b.step(1)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert np.array_equal(a.forces(7, 21), b.forces(7, 21))
    a.close()
    b.close()


def test_wall_2103296_full_size_step():
    """The 2,103,296-node mesh round the cylinder of the bounded unstructured
    workload (D 640, far field 8 D, Ma 0.2, Re 1000), launched as the
    benchmark launches it: one step against the oracle (populations and the
    force record)."""
    case = q9_cylinder_case(512, 640.0, 8.0, seed=1, Ma=0.2, Re=1000.0)
    sim, ora = paired(case)
    sim.step(1)
    ora.step()
    f, g = sim.populations()
    for a, b in ((f[:, 0, :], ora.f), (g[:, 0, :], ora.g)):
        err = np.abs(a - b)
        assert np.max(err) <= 1e-6 * np.max(np.abs(b)), (np.unravel_index(np.argmax(err), err.shape),
                                                         np.max(err))
    # the load on the new populations (record of level 1): 1e-4 of the load
    # plus the FP32 rounding of a pressure sum round the wall (1e-7 p pi D)
    h = sim.forces(1, 1)[0]
    Fx, Fy, _ = ora.wall_force()
    floor = 1e-7 * (1.0 / 3.0) * np.pi * 640.0
    assert abs(h[1] - Fx) <= 1e-4 * abs(Fx) + floor and abs(h[2] - Fy) <= 1e-4 * abs(Fy) + floor


def test_wall_device_gathers_agree_with_the_block_path(monkeypatch):
    """Round a body too, the interpolation through device memory
    (FSILBM_UNSTRUCTURED_GATHER=device) and the LDS-staged block path agree
    to FP32 rounding (missing populations take a placeholder in both, which
    the wall and far-field kernels replace)."""
    from paper_2107_01370_amd.fsilbm import Simulation
    mesh, fl, body, (rho, ux, uy, T) = q9_cylinder_case(seed=6)
    out = []
    for mode in (None, "device"):
        if mode:
            monkeypatch.setenv("FSILBM_UNSTRUCTURED_GATHER", mode)
        else:
            monkeypatch.delenv("FSILBM_UNSTRUCTURED_GATHER", raising=False)
        sim = Simulation(mesh, fl, [body])
        sim.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        sim.step(30)
        out.append((sim.populations(), sim.forces(0, 31)))
        sim.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))
    fs = np.max(np.hypot(out[1][1][:, 1], out[1][1][:, 2]))
    assert np.max(np.abs(out[0][1][:, 1:3] - out[1][1][:, 1:3])) <= 1e-4 * fs


def paired_moving(case):
    from paper_2107_01370_amd.fsilbm import Simulation
    mesh, fl, body, (rho, ux, uy, T) = case
    sim = Simulation(mesh, fl, [body])
    sim.init_equilibrium(rho[None], ux[None], uy[None], T[None])
    f0, g0 = sim.populations()
    ora = UnstructuredWallSolver(mesh, fl, body, rho, ux, uy, T)
    ora.f = f0[:, 0, :].astype(np.float64)
    ora.g = g0[:, 0, :].astype(np.float64)
    return sim, ora


def test_heaving_body_one_step_population_parity():
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case())
    sim.step(1)
    ora.step()
    f, g = sim.populations()
    for a, b in ((f[:, 0, :], ora.f), (g[:, 0, :], ora.g)):
        err = np.abs(a - b)
        assert np.max(err) <= 1e-6 * np.max(np.abs(b)), (np.unravel_index(np.argmax(err), err.shape),
                                                         np.max(err))


@pytest.mark.parametrize("dof", [0, 1])
def test_moving_body_60_steps_fields_forces_motion(dof):
    """Prescribed heave (dof 0) and a cylinder released on a spring (dof 1)
    on the blended unstructured mesh: fields, loads and the body's motion
    against the oracle."""
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case(seed=2, dof=dof))
    n = 60
    sim.step(n)
    ora.run(n)
    rho, ux, uy, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale
    amp = np.max(np.abs(ho[:, 4] - ho[0, 4]))
    assert amp > 0 and np.max(np.abs(hist[:, 4] - ho[:, 4])) <= 1e-4 * amp


def test_heaving_body_symmetric_mesh_has_no_cross_force():
    from synth.unstructured import q9_heave_case
    sim, _ = paired_moving(q9_heave_case(symmetric=True))
    sim.step(60)
    h = sim.forces(0, 61)
    assert abs(h[-1, 2]) > 0.1
    assert np.max(np.abs(h[:, 1])) <= 1e-4 * np.max(np.abs(h[:, 2]))


def test_heaving_cylinder_in_a_stream():
    """Prescribed heave across a free stream (the moving mesh, the wall's
    mesh velocity and the far field together): fields and loads against the
    oracle after 40 steps."""
    from synth.unstructured import q9_cylinder_case
    sim, ora = paired_moving(q9_cylinder_case(32, 40.0, 6.0, seed=3, Ma=0.2, Re=200.0, heave_D=0.1))
    n = 40
    sim.step(n)
    ora.run(n)
    rho, _, _, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale
    assert np.max(np.abs(hist[:, 4] - ho[:, 4])) <= 1e-9 * 4.0


def test_pitching_and_heaving_body_about_an_offset_axis():
    """Prescribed pitch about an elastic axis a quarter diameter off the
    centre, with heave: the rigid zone rotates, so g = R(alpha) there and
    the wall moves tangentially; fields, loads and the moment against the
    oracle after 40 steps."""
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case(seed=4, pitch_deg=2.0, ea_D=0.25))
    n = 40
    sim.step(n)
    ora.run(n)
    rho, _, _, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale
    mscale = np.max(np.abs(ho[:, 3]))
    assert mscale > 0 and np.max(np.abs(hist[:, 3] - ho[:, 3])) <= 1e-4 * mscale
    assert np.max(np.abs(hist[:, 5] - ho[:, 5])) <= 1e-12


def test_moving_body_fp16_storage_within_2e3():
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case(seed=5, storage=1))
    n = 20
    sim.step(n)
    ora.run(n)
    rho, _, _, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 2e-3
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 2e-3


def test_moving_body_checkpoint_and_single_steps_keep_the_run():
    """A moving body's checkpoint carries the departure table each step's
    relocation starts from: a fresh context loaded from it, stepped one step
    at a time, repeats the original run bitwise (16-step graphs there)."""
    from paper_2107_01370_amd.fsilbm import Simulation
    from synth.unstructured import q9_heave_case
    mesh, fl, body, (rho, ux, uy, T) = q9_heave_case(seed=6)

    def fresh():
        s = Simulation(mesh, fl, [body])
        s.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        return s

    a = fresh()
    a.step(7)
    ckpt = a.save()
    a.step(20)
    b = fresh()
    b.step(3)                      # a different departure table before the load
    b.load(ckpt)
    for _ in range(20):
        b.step(1)
    fa, ga = a.populations()
    fb, gb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert np.array_equal(a.forces(7, 21), b.forces(7, 21))
    a.close()
    b.close()


def test_moving_body_with_distance_blending():
    """Heave with the blending measured from the wall polygon (distances D/4
    and 2D): fields, loads and motion against the oracle after 40 steps."""
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case(seed=7, distance_blend=True))
    n = 40
    sim.step(n)
    ora.run(n)
    rho, _, _, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale


def test_body_carried_by_uniform_gas_changes_nothing_but_its_position():
    """The Galilean check on the device: the gas stays uniform to FP32
    rounding, the load stays at rounding level against p times the
    perimeter, the body moves at the gas velocity, and the oracle agrees."""
    from synth.unstructured import q9_comoving_case
    sim, ora = paired_moving(q9_comoving_case())
    mesh, fl = sim.mesh, ora.fluid
    n = 30
    sim.step(n)
    ora.run(n)
    rho, ux, uy, T = sim.macro()
    U = fl.u_inf[1]
    assert np.max(np.abs(rho[0] - 1.0)) <= 1e-6 and np.max(np.abs(ux[0])) <= 1e-6
    assert np.max(np.abs(uy[0] - U)) <= 1e-6 and np.max(np.abs(T[0] - fl.T_inf)) <= 1e-6
    hist = sim.forces(0, n)
    perimeter = np.pi * 20.0
    assert np.max(np.abs(hist[:, 1:3])) <= 1e-5 * fl.rho_inf * fl.T_inf * perimeter
    assert abs(hist[-1, 4] - (n - 1) * fl.dt * U) <= 1e-9
    ho = np.array(ora.history)
    assert np.max(np.abs(hist[:, 4] - ho[:, 4])) <= 1e-12


def test_moving_body_device_gathers_agree_with_the_block_path(monkeypatch):
    """A moving body: the node-block kernel with the relocation folded in and
    the device-memory path with the relocation as a kernel of its own agree
    to FP32 rounding."""
    from paper_2107_01370_amd.fsilbm import Simulation
    from synth.unstructured import q9_heave_case
    mesh, fl, body, (rho, ux, uy, T) = q9_heave_case(seed=8)
    out = []
    for mode in (None, "device"):
        if mode:
            monkeypatch.setenv("FSILBM_UNSTRUCTURED_GATHER", mode)
        else:
            monkeypatch.delenv("FSILBM_UNSTRUCTURED_GATHER", raising=False)
        sim = Simulation(mesh, fl, [body])
        sim.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        sim.step(30)
        out.append((sim.populations(), sim.forces(0, 31)))
        sim.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))
    fs = np.max(np.hypot(out[1][1][:, 1], out[1][1][:, 2]))
    assert np.max(np.abs(out[0][1][:, 1:3] - out[1][1][:, 1:3])) <= 1e-4 * fs
    assert np.array_equal(out[0][1][:, 4], out[1][1][:, 4])


def test_moving_body_kernel_timing_keeps_the_run():
    """Timing the kernels of a moving body's step (repeated launches that
    leave the departure points alone) and restoring the moments leaves the
    run bitwise as it was."""
    from paper_2107_01370_amd.fsilbm import Simulation
    from synth.unstructured import q9_heave_case
    mesh, fl, body, (rho, ux, uy, T) = q9_heave_case(seed=9)
    runs = []
    for timed in (False, True):
        s = Simulation(mesh, fl, [body])
        s.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        s.step(7)
        if timed:
            s.time_kernels(3)
        s.step(12)
        runs.append((s.populations(), s.forces(0, 20)))
        s.close()
    (fa, ga), ha = runs[0]
    (fb, gb), hb = runs[1]
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb) and np.array_equal(ha, hb)


def test_strong_coupling_on_a_moving_unstructured_body():
    """Sub-iterations (four passes, relaxation 0.7) for a light cylinder on a
    spring on the moving unstructured mesh: fields, loads and motion against
    the oracle's strong coupling after 30 steps."""
    from synth.unstructured import q9_heave_case
    sim, ora = paired_moving(q9_heave_case(seed=10, dof=1, mstar=0.5))
    sim.set_coupling(4, 0.7)
    ora.coupling(4, 0.7)
    n = 30
    sim.step(n)
    ora.run(n)
    rho, _, _, T = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    assert np.max(np.abs(rho[0] - r_o) / r_o) <= 1e-5
    assert np.max(np.abs(rho[0] * T[0] - r_o * T_o) / (r_o * T_o)) <= 1e-5
    hist = sim.forces(0, n)
    ho = np.array(ora.history)
    fscale = np.max(np.hypot(ho[:, 1], ho[:, 2]))
    assert np.max(np.abs(hist[:, 1:3] - ho[:, 1:3])) <= 1e-4 * fscale
    amp = np.max(np.abs(ho[:, 4] - ho[0, 4]))
    assert amp > 0 and np.max(np.abs(hist[:, 4] - ho[:, 4])) <= 1e-4 * amp


def test_fixed_body_subiterations_repeat_the_unstructured_step_bitwise():
    """Round a fixed body every pass streams the same populations onto the
    same mesh: with the level-n moments and wall values formed again before
    each pass, three passes give the staggered step bitwise."""
    from paper_2107_01370_amd.fsilbm import Simulation
    mesh, fl, body, (rho, ux, uy, T) = q9_cylinder_case(seed=11)
    out = []
    for passes in (1, 3):
        s = Simulation(mesh, fl, [body])
        s.set_coupling(passes, 0.7 if passes > 1 else 1.0)
        s.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        s.step(20)
        out.append((s.populations(), s.forces(0, 21)))
        s.close()
    (fa, ga), ha = out[0]
    (fb, gb), hb = out[1]
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb) and np.array_equal(ha, hb)


def test_mesh_read_from_a_gmsh_file_runs_like_the_original(tmp_path):
    """A moving-body mesh written as Gmsh MSH 2.2 and read back (elements
    re-oriented if needed, the wall loop assembled from its lines) gives the
    same populations bitwise and the same loads to FP64 summation order."""
    from paper_2107_01370_amd.fsilbm import Simulation
    from paper_2107_01370_amd.meshio import read_msh, write_msh
    from synth.unstructured import q9_heave_case
    mesh, fl, body, (rho, ux, uy, T) = q9_heave_case(seed=12)
    path = tmp_path / "heave.msh"
    write_msh(str(path), mesh)
    back = read_msh(str(path))
    assert np.array_equal(back.X, mesh.X) and np.array_equal(back.Y, mesh.Y)
    out = []
    for m in (mesh, back):
        s = Simulation(m, fl, [body])
        s.init_equilibrium(rho[None], ux[None], uy[None], T[None])
        s.step(20)
        out.append((s.populations(), s.forces(0, 21)))
        s.close()
    (fa, ga), ha = out[0]
    (fb, gb), hb = out[1]
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    assert np.max(np.abs(ha[:, 1:4] - hb[:, 1:4])) <= 1e-12 * np.max(np.abs(ha[:, 1:4]))
    assert np.array_equal(ha[:, 4], hb[:, 4])
