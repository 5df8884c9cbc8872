"""Pins of the oracle's surface-density block (Sec. 2.2.4: the orbit library's
surface mass in each aperture, converted to surface luminosity by the
stellar mass-to-light ratio Upsilon).

The block counts every mirror-copy event whose sky position falls in an
aperture, whatever its line-of-sight velocity.  Pins: with a velocity range
that holds every velocity it equals the kinematic block summed over the
velocity bins of each aperture; it does not change when the velocity bins
do; a brute-force recount of an orbit's trajectory through bin_points gives
the same counts; Upsilon divides that block and nothing else; with the block
off the matrix is the one without it.
"""
import numpy as np

import oracle as O
import workloads as W

CFG = W.SMALL
N_STEPS = 400


def _spec(**kw):
    s = dict(CFG["obs"])
    s.update(surface=1, upsilon=2.5)
    s.update(kw)
    return s


def _run(spec, n=48):
    ics, dt = W.grid_ics(W.load_table(CFG["table"]), seed=CFG["ic_seed"], n_steps=N_STEPS)
    pot = O.make_pot(CFG["components"], CFG["omega"])
    obs = O.make_obs(spec, O.euler_matrix(*CFG["euler"]))
    c, ov, _, _ = O.integrate_and_bin(pot, obs, ics[:, :n], dt[:n], N_STEPS)
    return obs, c, ov, ics[:, :n], dt[:n], pot


def _blocks(obs):
    nm = obs.nx * obs.ny * obs.nz
    nk = obs.n_ap * obs.nv
    return nm, nk


def test_wide_velocity_range_surface_is_aperture_sum():
    obs, c, _, _, _, _ = _run(_spec(vlo=-1e5, vhi=1e5))
    nm, nk = _blocks(obs)
    assert c.shape[1] == nm + nk + obs.n_ap
    kin = c[:, nm:nm + nk].reshape(c.shape[0], obs.n_ap, obs.nv).sum(2)
    assert np.array_equal(c[:, nm + nk:], kin)
    assert c[:, nm + nk:].sum() > 0


def test_surface_block_does_not_depend_on_velocity_bins():
    _, wide, _, _, _, _ = _run(_spec(vlo=-1e5, vhi=1e5))
    obs, narrow, ov, _, _, _ = _run(_spec(vlo=-50.0, vhi=50.0, nv=4))
    nm, nk = _blocks(obs)
    sig_w = wide[:, -obs.n_ap:]
    assert np.array_equal(narrow[:, nm + nk:], sig_w)
    kin = narrow[:, nm:nm + nk].reshape(narrow.shape[0], obs.n_ap, obs.nv).sum(2)
    assert np.all(kin <= sig_w) and (kin < sig_w).any()
    # the kinematic overflow counts the events outside the apertures or the velocity range
    assert np.array_equal(ov[:, 1], 4 * N_STEPS - kin.sum(1))


def test_brute_force_recount_from_the_trajectory():
    obs, c, _, ics, dt, pot = _run(_spec(vlo=-50.0, vhi=50.0, nv=4), n=6)
    nm, nk = _blocks(obs)
    for i in range(ics.shape[1]):
        traj = O.orbit(pot, ics[:, i], dt[i], N_STEPS)[1:]
        _, kin = O.bin_points(obs, np.ascontiguousarray(traj.T))
        k = kin.ravel()
        ap = np.where(k < 0, -1, np.where(k < nk, k // obs.nv, k - nk))
        want = np.bincount(ap[ap >= 0], minlength=obs.n_ap)
        assert np.array_equal(c[i, nm + nk:], want)
        assert np.array_equal(c[i, nm:nm + nk], np.bincount(k[(k >= 0) & (k < nk)], minlength=nk))


def test_upsilon_divides_the_surface_block_only():
    obs, c, _, _, _, _ = _run(_spec())
    A = O.time_fractions(c, N_STEPS, obs=obs)
    B = O.time_fractions(c, N_STEPS)
    nm, nk = _blocks(obs)
    assert np.array_equal(A[:, :nm + nk], B[:, :nm + nk])
    assert np.array_equal(A[:, nm + nk:], B[:, nm + nk:] / 2.5)


def test_block_off_gives_the_matrix_without_it():
    _, on, ov_on, _, _, _ = _run(_spec(surface=1))
    obs, off, ov_off, _, _, _ = _run(_spec(surface=0))
    assert off.shape[1] == on.shape[1] - obs.n_ap
    assert np.array_equal(off, on[:, :off.shape[1]]) and np.array_equal(ov_on, ov_off)
