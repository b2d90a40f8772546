"""The transport inputs of the disc generator (CPU): the faces put the cell
centres where make_cells has them, for every configuration shape, and the
dust and gas velocities have the frames the transport step takes."""
import numpy as np
import pytest

from paper_2402_18471_amd import disc


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (24, 12), (64, 32)])
def test_faces_centre_the_generator_cells(shape):
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], *shape, 12)
    R_e, t_e = disc.transport_grid(cfg)
    assert R_e.shape == (cfg.n_r + 1,) and t_e.shape == (cfg.n_z + 1,)
    assert t_e[0] == 0.0 and np.all(np.diff(R_e) > 0) and np.all(np.diff(t_e) > 0)
    cells = disc.make_cells(cfg)
    Rc = np.sqrt(R_e[:-1] * R_e[1:])
    tc = 0.5 * (t_e[:-1] + t_e[1:])
    R = cells["R"].reshape(cfg.n_r, cfg.n_z)
    Z = cells["Z"].reshape(cfg.n_r, cfg.n_z)
    assert np.allclose(R, Rc[:, None], rtol=1e-14, atol=0)
    assert np.allclose(Z, tc[None, :] * Rc[:, None], rtol=1e-14, atol=0)


def test_velocity_frames():
    cfg = disc.scaled(disc.CONFIGS["disc64x32_n100"], 8, 4, 10)
    s = np.geomspace(cfg.s_min, cfg.s_max, 10)
    d = disc.make_transport(cfg, s)
    R = d["cells"]["R"]
    v_k = np.sqrt(d["GM"] / R)
    # absolute azimuthal dust speed = Keplerian + the generator's lag; the
    # radial and vertical components as the coagulation inputs have them
    assert np.allclose(d["v"][:, :, 1], v_k[:, None] + d["v_dust"][:, :, 1], rtol=1e-15, atol=0)
    assert np.array_equal(d["v"][:, :, 0], d["v_dust"][:, :, 0])
    assert np.array_equal(d["v"][:, :, 2], d["v_dust"][:, :, 2])
    # the gas at rest in R and Z, rotating slightly below Omega R
    assert np.all(d["v_gas"][:, 0] == 0) and np.all(d["v_gas"][:, 2] == 0)
    om_r = d["cells"]["Omega"] * R
    assert np.all(d["v_gas"][:, 1] > 0.9 * om_r) and np.all(d["v_gas"][:, 1] < 1.1 * om_r)
