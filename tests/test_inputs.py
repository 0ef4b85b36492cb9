"""The seeded synthetic input generators (CPU): determinism and the properties
the workloads rely on."""
import numpy as np

import inputs


def test_plate_velocity_is_tangential_piecewise_rigid_and_seeded():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2000, 3))
    x /= np.linalg.norm(x, axis=1)[:, None]
    u = inputs.plate_velocity(13, x)
    assert np.abs(np.einsum("ij,ij->i", u, x)).max() < 1e-14          # u . n = 0 on the sphere
    assert np.array_equal(u, inputs.plate_velocity(13, x))              # seeded
    assert not np.allclose(u, inputs.plate_velocity(14, x))
    # rigid rotation per plate: u = omega_k x X for one of n_plates poles
    centres = np.random.default_rng(13).normal(size=(6, 3))
    centres /= np.linalg.norm(centres, axis=1)[:, None]
    plate = np.argmax(x @ centres.T, axis=1)
    for k in range(6):
        sel = plate == k
        if sel.sum() < 3:
            continue
        # one rotation vector om with u = om x X fits every point of the plate
        P = x[sel]
        C = np.zeros((len(P), 3, 3))                 # C @ om = X x om = -(om x X)
        C[:, 0, 1], C[:, 0, 2] = -P[:, 2], P[:, 1]
        C[:, 1, 0], C[:, 1, 2] = P[:, 2], -P[:, 0]
        C[:, 2, 0], C[:, 2, 1] = -P[:, 1], P[:, 0]
        om = np.linalg.lstsq(C.reshape(-1, 3), -u[sel].ravel(), rcond=None)[0]
        assert np.abs(np.cross(om, P) - u[sel]).max() < 1e-12


def test_base_viscosity_profile_is_positive_and_layered():
    b = inputs.base_viscosity_profile(65)
    r = np.linspace(inputs.R_IN, inputs.R_OUT, 65)
    assert (b > 0).all() and b.max() / b.min() > 1e2
    assert b[r >= 0.97].min() > b[(r > 0.88) & (r < 0.95)].max()         # stiff lithosphere over a weak layer


def test_splitmix64_matches_its_published_outputs():
    """The generator's widely reproduced reference sequence for the start
    state 1234567, and the mapping of the top 53 bits to [-1, 1)."""
    assert inputs.splitmix64(1234567, 5) == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                             4593380528125082431, 16408922859458223821]
    u = inputs.splitmix64_uniform(1234567, 5)
    assert np.allclose(u, [(z >> 11) / 2.0 ** 52 - 1.0 for z in inputs.splitmix64(1234567, 5)], rtol=0, atol=0)
    assert (u >= -1).all() and (u < 1).all()


def test_viscosity_1e6_reaches_its_contrast_with_depth_slab_and_temperature():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20000, 3))
    x = d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(0.55, 1.0, 20000)[:, None]
    T = inputs.SHField(2).temperature(x)
    eta = inputs.viscosity_1e6(x, T)
    assert abs(np.log(eta.max() / eta.min()) - np.log(1e6)) < 1e-9
    # depth: at fixed T outside the slab eta falls by 100 from r_in to r_out
    e2 = inputs.viscosity_1e6(np.array([[0.55, 0, 0], [1.0, 0, 0], [0.3, 0.4, 0.1]]), np.array([0.5, 0.5, 0.2]))
    assert np.isclose(e2[0] / e2[1], 100.0)
