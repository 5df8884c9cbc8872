"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/schw.h is exported by libschw.so, the structs have the same layout in C
and in the ctypes binding, and invalid arguments are rejected on the host,
before any device work, with the documented status codes."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2607_00117_amd as P
from paper_2607_00117_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "schw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return", "sizeof")))


def test_every_declared_symbol_is_exported():
    L = P.load()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "schw.h"\nint main(void){\n'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(sw_component), sizeof(sw_potential_desc),'
                   ' sizeof(sw_potential), sizeof(sw_obs_spec), sizeof(sw_solve_opts), sizeof(sw_solve_report),'
                   ' offsetof(sw_obs_spec, pix2ap), offsetof(sw_solve_opts, mask));\nreturn 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(_lib.Component), C.sizeof(_lib.PotentialDesc), C.sizeof(_lib.Potential),
            C.sizeof(_lib.ObsSpec), C.sizeof(_lib.SolveOpts), C.sizeof(_lib.SolveReport),
            _lib.ObsSpec.pix2ap.offset, _lib.SolveOpts.mask.offset]
    assert got == want


def test_build_potential_validation():
    P.build_potential([("plummer", (1e10, 0.5)), ("mn", (5e10, 3.0, 0.3))], 0.0, (0.1, 0.2, 0.3))
    P.build_potential([("da_t3", (1e10, 1.5, 0.6, 3.5, 0.4)), ("da_v4", (3e9, 0.0, 0.8, 2.0, -1.0))], 40.0)
    bad = [
        [("plummer", (-1.0, 0.5))],
        [("plummer", (1e10, 0.0))],
        [("mn", (1e10, -1.0, 0.3))],
        [("nfw_q", (1e12, 10.0, 0.0, 70.0))],
        [("ferrers2", (1e10, 4.0, 0.0, 1.0))],
        [(99, (1.0,))],
        [("kepler", (float("nan"),))],
        [("da_t3", (1e10, 1.0, 0.5, 3.0, 1.5))],   # eta outside [-1, 1]
        [("da_v4", (1e10, 1.0, 0.5, 0.0, 0.0))],   # L = 0
        [("da_t3", (1e10, 1.0, 0.0, 3.0, 0.0))],   # b = 0
        [("da_v4", (1e10, -1.0, 0.5, 3.0, 0.0))],  # a < 0
    ]
    for comps in bad:
        with pytest.raises(P.SchwError) as e:
            P.build_potential(comps)
        assert e.value.status == -1
    with pytest.raises(P.SchwError):
        P.build_potential([("kepler", (1.0,))], float("inf"))
    d = _lib.PotentialDesc()
    d.n_comp = 9  # more than SW_MAX_COMP
    assert P.load().build_potential(C.byref(d), C.byref(_lib.Potential())) == -1


def _obs():
    return P.obs_spec(dict(nx=4, ny=4, nz=2, lo=(-1, -1, -1), hi=(1, 1, 1), npx=2, npy=2, plo=(-1, -1), phi=(1, 1),
                           nv=3, vlo=-1, vhi=1, symmetrize=1, drift_every=1))


def test_integrate_and_bin_validation_before_launch():
    L = P.load()
    pot = P.build_potential([("kepler", (1e10,))])
    obs = _obs()
    arr = (_lib.Potential * 1)(pot)
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first

    def call(n_pot=1, offs=(0, 10), n=10, steps=5, dtype=1, obs_=obs, ws=1 << 20):
        o = (C.c_int64 * len(offs))(*offs)
        return L.integrate_and_bin(arr, n_pot, o, fake, fake, n, steps, dtype, C.byref(obs_), fake, fake, fake, fake,
                                   fake, ws, None)
    assert call(dtype=3) == -1
    assert call(offs=(0, 9)) == -1          # offsets must end at n_orb
    assert call(steps=0) == -1
    assert call(n_pot=0) == -1
    bad = _obs()
    bad.nx = 0
    assert call(obs_=bad) == -1
    big = _obs()
    big.nx, big.ny, big.nz = 100, 100, 100    # mass block beyond 16-bit cell indices
    assert call(obs_=big) == -1
    assert call(ws=16) == -2                # workspace too small
    assert b"workspace" in L.sw_last_error()


def test_cell_masses_validation_before_launch():
    L = P.load()
    pot = P.build_potential([("mn", (5e10, 3.0, 0.3)), ("ferrers2", (1e10, 4.0, 1.5, 1.0)),
                             ("nfw_q", (1e12, 10.0, 0.9, 70.0)), ("kepler", (1e8,))])
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first

    def call(mask=0b11, n_sub=4, obs_=None, out=fake):
        return L.cell_masses(C.byref(pot), C.byref(obs_ or _obs()), mask, n_sub, out, None)
    assert call(mask=0) == -1                 # nothing selected
    assert call(mask=0b10000) == -1           # component 4 does not exist
    assert call(mask=0b111) == -1             # the NFW halo has no stellar density
    assert call(mask=0b1001) == -1            # nor has a point mass
    assert b"no stellar density" in L.sw_last_error()
    assert call(n_sub=0) == -1 and call(n_sub=17) == -1
    assert call(out=None) == -1
    bad = _obs()
    bad.nz = 0
    assert call(obs_=bad) == -1
    cyl = _obs()
    cyl.grid = P.SW_GRID_CYLINDRICAL
    cyl.lo[0] = -1.0                          # R must start at >= 0
    assert call(obs_=cyl) == -1


def test_jeans_ics_validation_before_launch():
    L = P.load()
    pot = P.build_potential([("mn", (5e10, 3.0, 0.3))])
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first

    def call(n=4, hR=3.5, hz=1.2, b=1.0, out=fake):
        return L.jeans_ics(C.byref(pot), fake, fake, n, hR, hz, b, fake, out, None)
    assert call(n=-1) == -1
    assert call(hR=0.0) == -1 and call(hz=float("nan")) == -1
    assert call(b=0.0) == -1
    assert call(out=None) == -1
    assert call(n=0, out=None) == 0          # nothing to do
    assert L.dither_ics(fake, fake, fake, 4, 0, 0.1, 0.05, fake, None) == -1   # no realisations
    assert L.dither_ics(fake, fake, fake, 4, 4, -0.1, 0.05, fake, None) == -1  # negative box
    assert L.bundle_rows(fake, 3, 2, 5, 4, fake, None) == -1                   # dtype
    assert L.bundle_rows(fake, 1, 2, 5, 4, fake, None) == -1                   # aliased
    assert L.bundle_rows(fake, 1, 2, 5, 0, C.c_void_p(0x2000), None) == -1     # n_dither = 0


def test_solve_and_chi2_validation_before_launch():
    L = P.load()
    opts = _lib.SolveOpts()
    opts.gram, opts.nu = 1, 1e-2
    fake = C.c_void_p(0x1000)
    rep = _lib.SolveReport()
    assert L.solve_weights(fake, 1, 100, 50, fake, fake, 1.0, -1.0, C.byref(opts), fake, C.byref(rep), fake, 16,
                           None) == -2
    assert L.solve_weights(fake, 1, 100, 50, fake, fake, 0.0, -1.0, C.byref(opts), fake, C.byref(rep), fake, 1 << 40,
                           None) == -1  # w_tilde must be > 0
    opts.gram = 7
    assert L.solve_weights(fake, 1, 100, 50, fake, fake, 1.0, -1.0, C.byref(opts), fake, C.byref(rep), fake, 1 << 40,
                           None) == -1
    out = C.c_double()
    assert L.chi2(fake, 1, 10, 5, fake, fake, fake, 3, 9, C.byref(out), fake, 1 << 20, None) == -1  # range > n_con
    assert P.solve_workspace_bytes(0, 10, opts) == 0
    assert P.chi2_workspace_bytes(100) > 0


def test_chi2_noalloc_validation_before_launch():
    """The no-allocation chi2 rejects sizes beyond its static scratch and bad
    arguments on the host, before touching the device."""
    L = P.load()
    fake = C.c_void_p(0x1000)
    out = C.c_double()
    lim = P.chi2_noalloc_max_con()
    assert lim == 65536
    assert L.chi2_noalloc(fake, 1, 10, lim + 1, fake, fake, fake, 0, 5, C.byref(out), None) == -1
    assert "static scratch limit" in L.sw_last_error().decode()
    assert L.chi2_noalloc(fake, 1, 10, 5, fake, fake, fake, 3, 9, C.byref(out), None) == -1  # range > n_con
    assert L.chi2_noalloc(fake, 3, 10, 5, fake, fake, fake, 0, 5, C.byref(out), None) == -1  # dtype
    assert L.chi2_noalloc(None, 1, 10, 5, fake, fake, fake, 0, 5, C.byref(out), None) == -1  # null matrix


def test_workspace_queries_scale():
    obs = _obs()
    a = P.integrate_workspace_bytes(obs, 1, 1000, 100, 1)
    b = P.integrate_workspace_bytes(obs, 1, 2000, 100, 1)
    assert b > a >= 2 * 1000 * 100 * 8
    opts = _lib.SolveOpts()
    opts.gram = 1
    s1 = P.solve_workspace_bytes(1000, 300, opts)
    s2 = P.solve_batched_workspace_bytes([0, 500, 1000], 300, opts)
    assert s1 > 0 and s2 > 0


def test_tuning_knobs():
    assert P.get_tuning("hist_lds_kb") > 0
    with pytest.raises(P.SchwError):
        P.set_tuning("hist_lds_kb", 1000)
    with pytest.raises(P.SchwError):
        P.set_tuning("no_such_knob", 1)
    assert P.get_tuning("no_such_knob") == -1
    old = P.get_tuning("hist_lds_kb")
    P.set_tuning("hist_lds_kb", 32)
    assert P.get_tuning("hist_lds_kb") == 32
    P.set_tuning("hist_lds_kb", old)
    # every knob: its default reads back, an out-of-range value is refused and leaves it unchanged
    for key, good, bad in [("integrate_waves_per_cu", 8, 65), ("integrate_lanes_per_orbit", 2, 3),
                           ("sparse_rows_per_wg", 64, 17), ("sparse_cols_per_wg", 512, 1024),
                           ("sparse_lanes_per_row", 16, 32), ("rhs_per_group", 4, 3)]:
        old = P.get_tuning(key)
        assert old >= 0
        P.set_tuning(key, good)
        assert P.get_tuning(key) == good
        with pytest.raises(P.SchwError):
            P.set_tuning(key, bad)
        assert P.get_tuning(key) == good
        P.set_tuning(key, old)


def test_mlp_param_count_matches_architecture():
    assert P.mlp_param_count() == 256 * 12 + 256 + 2 * (256 * 256 + 256) + 256 + 1
    assert P.mlp_workspace_bytes(0) == 0
