"""ctypes binding of libschw.so (see include/schw.h for every entry point's contract).

Arguments that are device buffers are passed as torch tensors on the current
HIP device (their data pointers are handed to the library); the stream is
torch's current stream.  Nothing here computes: it validates dtypes/shapes
only as far as needed to pass pointers, and raises SchwError on a non-zero
status.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))

SW_F32, SW_F64 = 1, 2
SW_GRAM_BF16, SW_GRAM_BF16X3, SW_GRAM_F32 = 0, 1, 2
SW_SOLVE_DENSE = 1
SW_SOLVE_NO_ACCEL = 2
SW_FLAG_DRIFT, SW_FLAG_NONFINITE = 1, 2
SW_GRID_CARTESIAN, SW_GRID_CYLINDRICAL = 0, 1
KINDS = {"kepler": 1, "isochrone": 2, "plummer": 3, "mn": 4, "nfw_q": 5, "ferrers2": 6, "da_t3": 7, "da_v4": 8}


class SchwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Component(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("p", C.c_double * 8)]


class PotentialDesc(C.Structure):
    _fields_ = [("n_comp", C.c_int32), ("reserved", C.c_int32), ("comp", Component * 8),
                ("omega_b", C.c_double), ("euler", C.c_double * 3)]


class Potential(C.Structure):
    _fields_ = [("opaque", C.c_uint8 * 2048)]


class ObsSpec(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("grid", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("npx", C.c_int32), ("npy", C.c_int32), ("plo", C.c_double * 2), ("phi", C.c_double * 2),
                ("pix2ap", C.c_void_p), ("n_ap", C.c_int32), ("nv", C.c_int32),
                ("vlo", C.c_double), ("vhi", C.c_double),
                ("symmetrize", C.c_int32), ("drift_every", C.c_int32),
                ("surface", C.c_int32), ("pad", C.c_int32), ("upsilon", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("gram", C.c_int32), ("max_iter", C.c_int32), ("refine_iter", C.c_int32),
                ("check_every", C.c_int32), ("use_graph", C.c_int32), ("flags", C.c_int32),
                ("rho", C.c_double), ("tol", C.c_double),
                ("tol_kkt", C.c_double), ("nu", C.c_double), ("mask", C.c_void_p), ("w0", C.c_void_p),
                ("w0_shared", C.c_int32), ("reserved", C.c_int32), ("quantum", C.c_double)]


class SolveReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refine_iters", C.c_int32), ("converged", C.c_int32),
                ("n_active", C.c_int32), ("mu", C.c_double), ("rho", C.c_double), ("kkt", C.c_double),
                ("objective", C.c_double), ("primal_res", C.c_double), ("dual_res", C.c_double),
                ("t_prep_ms", C.c_double), ("t_gram_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_admm_ms", C.c_double), ("t_refine_ms", C.c_double), ("nnz", C.c_double),
                ("passes", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_L = None


def library_path():
    return os.path.join(HERE, "libschw.so")


def load():
    """Loads libschw.so; raises if it has not been built (no fallback)."""
    global _L
    if _L is not None:
        return _L
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2607_00117_amd/build.py "
                          "(or __graft_entry__.build()); there is no non-HIP fallback")
    L = C.CDLL(path)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.build_potential.argtypes = [C.POINTER(PotentialDesc), C.POINTER(Potential)]
    L.integrate_and_bin.argtypes = [C.POINTER(Potential), i32, C.POINTER(C.c_int64), vp, vp, i64, i32, i32,
                                    C.POINTER(ObsSpec), vp, vp, vp, vp, vp, sz, vp]
    L.integrate_workspace_bytes.argtypes = [C.POINTER(ObsSpec), i32, i64, i32, i32]
    L.integrate_workspace_bytes.restype = sz
    L.solve_weights.argtypes = [vp, i32, i64, i64, vp, vp, C.c_double, C.c_double, C.POINTER(SolveOpts), vp,
                                C.POINTER(SolveReport), vp, sz, vp]
    L.solve_workspace_bytes.argtypes = [i64, i64, C.POINTER(SolveOpts)]
    L.solve_workspace_bytes.restype = sz
    L.solve_weights_batched.argtypes = [vp, i32, i32, C.POINTER(C.c_int64), i64, vp, vp, C.POINTER(C.c_double),
                                        C.c_double, C.POINTER(SolveOpts), vp, C.POINTER(SolveReport), vp, sz, vp]
    L.solve_batched_workspace_bytes.argtypes = [i32, C.POINTER(C.c_int64), i64, C.POINTER(SolveOpts)]
    L.solve_batched_workspace_bytes.restype = sz
    L.solve_weights_multi.argtypes = [vp, i32, i64, i64, i32, vp, vp, C.c_double, C.c_double, C.POINTER(SolveOpts),
                                      vp, C.POINTER(SolveReport), vp, sz, vp]
    L.solve_multi_workspace_bytes.argtypes = [i64, i64, i32, C.POINTER(SolveOpts)]
    L.solve_multi_workspace_bytes.restype = sz
    L.bootstrap_data.argtypes = [vp, vp, vp, i64, i32, i64, i64, vp, vp]
    L.chi2_model.argtypes = [C.POINTER(C.c_double), i32, C.POINTER(C.c_double)]
    L.chi2.argtypes = [vp, i32, i64, i64, vp, vp, vp, i64, i64, C.POINTER(C.c_double), vp, sz, vp]
    L.chi2_workspace_bytes.argtypes = [i64]
    L.gh_fit_workspace_bytes.argtypes = [i32, i32, i32]
    L.gh_fit_workspace_bytes.restype = sz
    L.gh_fit_matrix.argtypes = [vp, i32, i64, i64, i64, i64, i64, i32, i32, C.c_double, C.c_double,
                                C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double), i32, vp, vp, sz, vp]
    L.chi2_noalloc.argtypes = [vp, i32, i64, i64, vp, vp, vp, i64, i64, C.POINTER(C.c_double), vp]
    L.chi2_noalloc_max_con.argtypes = []
    L.chi2_noalloc_max_con.restype = i64
    L.chi2_workspace_bytes.restype = sz
    L.model_observables.argtypes = [vp, i32, i64, i64, vp, vp, vp]
    L.bin_points.argtypes = [C.POINTER(Potential), C.POINTER(ObsSpec), vp, i64, i32, vp, vp, vp]
    L.cell_masses.argtypes = [C.POINTER(Potential), C.POINTER(ObsSpec), C.c_uint32, i32, vp, vp]
    L.jeans_ics.argtypes = [C.POINTER(Potential), vp, vp, i64, C.c_double, C.c_double, C.c_double, vp, vp, vp]
    L.dither_ics.argtypes = [vp, vp, vp, i64, i32, C.c_double, C.c_double, vp, vp]
    L.bundle_rows.argtypes = [vp, i32, i64, i64, i32, vp, vp]
    L.integrate_bs23_and_bin.argtypes = [C.POINTER(Potential), vp, vp, i64, i32, C.c_double, C.c_double, i32,
                                         C.POINTER(ObsSpec), vp, vp, vp, vp, vp, sz, vp]
    L.integrate_bs23_workspace_bytes.argtypes = [i64, i32]
    L.integrate_bs23_workspace_bytes.restype = sz
    L.integrate_orbits.argtypes = [C.POINTER(Potential), vp, vp, i64, i32, i32, vp, vp]
    L.mlp_param_count.restype = i64
    L.mlp_workspace_bytes.argtypes = [i64]
    L.mlp_workspace_bytes.restype = sz
    L.mlp_forward.argtypes = [vp, vp, i64, vp, vp, sz, vp]
    L.mlp_backward.argtypes = [vp, vp, i64, vp, vp, vp, sz, vp]
    L.mlp_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.mlp_pack_bf16.argtypes = [vp, vp, vp]
    L.mlp_mse_grad.argtypes = [vp, vp, i64, vp, vp]
    L.mlp_infer_bf16.argtypes = [vp, vp, i64, vp, vp]
    L.gh_workspace_bytes.argtypes = [i32, i32, i32]
    L.gh_workspace_bytes.restype = sz
    L.gh_moments.argtypes = [vp, i32, i64, i64, i64, i32, i32, C.c_double, C.c_double, C.POINTER(C.c_double),
                             C.POINTER(C.c_double), i32, vp, vp, sz, vp]
    L.sw_set_tuning.argtypes = [C.c_char_p, i32]
    L.sw_get_tuning.argtypes = [C.c_char_p]
    L.sw_get_tuning.restype = i32
    L.sw_last_error.restype = C.c_char_p
    _L = L
    return L


def _check(status):
    if status != 0:
        raise SchwError(status, load().sw_last_error().decode())
    return status


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return SW_F32
    if t.dtype == torch.float64:
        return SW_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def build_potential(components, omega=0.0, euler=(0.0, 0.0, 0.0)):
    """components: list of (kind name, params) in the slot order of include/schw.h."""
    d = PotentialDesc()
    d.n_comp = len(components)
    for i, (kind, params) in enumerate(components):
        d.comp[i].kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        for j, v in enumerate(params):
            d.comp[i].p[j] = float(v)
    d.omega_b = float(omega)
    for i in range(3):
        d.euler[i] = float(euler[i])
    out = Potential()
    _check(load().build_potential(C.byref(d), C.byref(out)))
    return out


def count_quantum(obs, n_steps):
    """opts.quantum for integrate_and_bin's output: its entries are counts of
    1 / (ncopy n_steps), ncopy = 4 with the mirror copies, else 1; 0 (off) with
    surface-density columns (divided by the mass-to-light ratio) or counts
    that may exceed 65535."""
    ncopy = 4 if obs.symmetrize else 1
    if obs.surface or ncopy * int(n_steps) > 65535:
        return 0.0
    return 1.0 / (ncopy * int(n_steps))


def obs_spec(spec, pix2ap=None):
    """spec: dict (nx, ny, nz, lo, hi, npx, npy, plo, phi, nv, vlo, vhi, symmetrize, drift_every,
    n_ap, optional grid, surface, upsilon); pix2ap: optional int32 device tensor."""
    o = ObsSpec()
    o.nx, o.ny, o.nz = spec["nx"], spec["ny"], spec["nz"]
    o.grid = 1 if spec.get("grid", "cartesian") == "cylindrical" else 0
    for i in range(3):
        o.lo[i], o.hi[i] = spec["lo"][i], spec["hi"][i]
    o.npx, o.npy = spec["npx"], spec["npy"]
    for i in range(2):
        o.plo[i], o.phi[i] = spec["plo"][i], spec["phi"][i]
    if pix2ap is not None:
        o.pix2ap = pix2ap.data_ptr()
        o._pix2ap = pix2ap  # the spec keeps the device map alive as long as it is used
        o.n_ap = int(spec["n_ap"])
    else:
        o.pix2ap = None
        o.n_ap = spec["npx"] * spec["npy"]
    o.nv, o.vlo, o.vhi = spec["nv"], spec["vlo"], spec["vhi"]
    o.symmetrize = int(spec.get("symmetrize", 1))
    o.drift_every = int(spec.get("drift_every", 1))
    o.surface = int(spec.get("surface", 0))
    o.upsilon = float(spec.get("upsilon", 1.0))
    return o


def ncon(obs):
    return obs.nx * obs.ny * obs.nz + obs.n_ap * obs.nv + (obs.n_ap if obs.surface else 0)


def _pots_array(pots):
    if isinstance(pots, Potential):
        pots = [pots]
    arr = (Potential * len(pots))(*pots)
    return arr, len(pots)


def integrate_workspace_bytes(obs, n_pot, n_orb, n_steps, dtype):
    return load().integrate_workspace_bytes(C.byref(obs), n_pot, n_orb, n_steps, dtype)


def integrate_and_bin(pots, offsets, ics, dt, n_steps, obs, A, overflow, drift, flags, workspace):
    arr, n_pot = _pots_array(pots)
    offs = (C.c_int64 * (n_pot + 1))(*[int(v) for v in offsets])
    n_orb = ics.shape[1]
    _check(load().integrate_and_bin(arr, n_pot, offs, _ptr(ics), _ptr(dt), n_orb, int(n_steps),
                                    _dtype_code(ics), C.byref(obs), _ptr(A), _ptr(overflow), _ptr(drift),
                                    _ptr(flags), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream()))


def solve_workspace_bytes(n_orb, n_con, opts):
    return load().solve_workspace_bytes(n_orb, n_con, C.byref(opts))


def solve_weights(A, d, sigma, w_tilde, lam, opts, w, workspace):
    rep = SolveReport()
    n_orb, n_con = A.shape
    st = load().solve_weights(_ptr(A), _dtype_code(A), n_orb, n_con, _ptr(d), _ptr(sigma), float(w_tilde),
                              float(lam), C.byref(opts), _ptr(w), C.byref(rep), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream())
    if st not in (0, -4):
        _check(st)
    return st, rep


def solve_batched_workspace_bytes(offsets, n_con, opts):
    offs = (C.c_int64 * len(offsets))(*[int(v) for v in offsets])
    return load().solve_batched_workspace_bytes(len(offsets) - 1, offs, n_con, C.byref(opts))


def solve_weights_batched(A, offsets, d, sigma, w_tilde, lam, opts, w, workspace):
    """d, sigma: device [n_prob][n_con]; w_tilde: sequence of n_prob floats."""
    n_prob = len(offsets) - 1
    offs = (C.c_int64 * (n_prob + 1))(*[int(v) for v in offsets])
    wt = (C.c_double * n_prob)(*[float(v) for v in w_tilde])
    reps = (SolveReport * n_prob)()
    st = load().solve_weights_batched(_ptr(A), _dtype_code(A), n_prob, offs, A.shape[1], _ptr(d), _ptr(sigma), wt,
                                      float(lam), C.byref(opts), _ptr(w), reps, _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream())
    if st not in (0, -4):
        _check(st)
    return st, list(reps)


def solve_multi_workspace_bytes(n_orb, n_con, n_rhs, opts):
    return load().solve_multi_workspace_bytes(int(n_orb), int(n_con), int(n_rhs), C.byref(opts))


def solve_weights_multi(A, d, sigma, w_tilde, lam, opts, w, workspace):
    """d: device [n_rhs][n_con]; sigma: device [n_con]; w: device [n_rhs][n_orb]."""
    n_orb, n_con = A.shape
    n_rhs = d.shape[0]
    reps = (SolveReport * n_rhs)()
    st = load().solve_weights_multi(_ptr(A), _dtype_code(A), n_orb, n_con, n_rhs, _ptr(d), _ptr(sigma),
                                    float(w_tilde), float(lam), C.byref(opts), _ptr(w), reps, _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), _stream())
    if st not in (0, -4):
        _check(st)
    return st, list(reps)


def bootstrap_data(d, sigma, eps, col_begin, col_end, out):
    """d, sigma: device [n_con]; eps, out: device [n_rhs][n_con]."""
    n_rhs, n_con = eps.shape
    _check(load().bootstrap_data(_ptr(d), _ptr(sigma), _ptr(eps), int(n_con), int(n_rhs), int(col_begin),
                                 int(col_end), _ptr(out), _stream()))


def chi2_model(chi2_b):
    vals = [float(v) for v in chi2_b]
    arr = (C.c_double * max(1, len(vals)))(*vals)
    out = C.c_double(0.0)
    _check(load().chi2_model(arr, len(vals), C.byref(out)))
    return out.value


def chi2_workspace_bytes(n_con):
    return load().chi2_workspace_bytes(n_con)


def chi2(A, w, d, sigma, col_begin, col_end, workspace):
    out = C.c_double(0.0)
    n_orb, n_con = A.shape
    _check(load().chi2(_ptr(A), _dtype_code(A), n_orb, n_con, _ptr(w), _ptr(d), _ptr(sigma), int(col_begin),
                       int(col_end), C.byref(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                       _stream()))
    return out.value


def chi2_noalloc(A, w, d, sigma, col_begin, col_end):
    out = C.c_double(0.0)
    n_orb, n_con = A.shape
    _check(load().chi2_noalloc(_ptr(A), _dtype_code(A), n_orb, n_con, _ptr(w), _ptr(d), _ptr(sigma), int(col_begin),
                               int(col_end), C.byref(out), _stream()))
    return out.value


def chi2_noalloc_max_con():
    return int(load().chi2_noalloc_max_con())


def gh_fit_workspace_bytes(n_ap, nv, n_gh=4):
    return load().gh_fit_workspace_bytes(int(n_ap), int(nv), int(n_gh))


def gh_fit_matrix(A, n_mass, kin0, surf0, n_ap, nv, vlo, vhi, v0, s, gamma, out, workspace, n_gh=4):
    """out: device [n_orb][n_mass (+ n_ap) + n_gh * n_ap] of A's dtype; surf0 < 0: no surface block;
    v0, s, gamma: sequences of n_ap floats."""
    n_orb, n_con = A.shape
    arr = lambda v: (C.c_double * n_ap)(*[float(x) for x in v])  # noqa: E731
    _check(load().gh_fit_matrix(_ptr(A), _dtype_code(A), n_orb, n_con, int(n_mass), int(kin0), int(surf0), int(n_ap),
                                int(nv), float(vlo), float(vhi), arr(v0), arr(s), arr(gamma), int(n_gh), _ptr(out),
                                _ptr(workspace), workspace.numel() * workspace.element_size(), _stream()))


def gh_workspace_bytes(n_ap, nv, n_gh=4):
    return load().gh_workspace_bytes(int(n_ap), int(nv), int(n_gh))


def gh_moments(A, kin0, n_ap, nv, vlo, vhi, v0, s, out, workspace, n_gh=4):
    """out: device [n_orb][n_ap][n_gh + 1] double; v0, s: sequences of n_ap floats."""
    n_orb, n_con = A.shape
    v0a = (C.c_double * n_ap)(*[float(v) for v in v0])
    sa = (C.c_double * n_ap)(*[float(v) for v in s])
    _check(load().gh_moments(_ptr(A), _dtype_code(A), n_orb, n_con, int(kin0), int(n_ap), int(nv), float(vlo),
                             float(vhi), v0a, sa, int(n_gh), _ptr(out), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream()))


def model_observables(A, w, out):
    n_orb, n_con = A.shape
    _check(load().model_observables(_ptr(A), _dtype_code(A), n_orb, n_con, _ptr(w), _ptr(out), _stream()))


def bin_points(pot, obs, pts, mass, kin):
    _check(load().bin_points(C.byref(pot), C.byref(obs), _ptr(pts), pts.shape[1], _dtype_code(pts), _ptr(mass),
                             _ptr(kin), _stream()))


def cell_masses(pot, obs, comp_mask, n_sub, out):
    """m*_n of the components selected by comp_mask into out (device double [n_mass])."""
    _check(load().cell_masses(C.byref(pot), C.byref(obs), int(comp_mask), int(n_sub), _ptr(out), _stream()))


def jeans_ics(pot, pos, eps, h_R, h_z, b, moments, ics):
    """Jeans-equation initial conditions at pos (device double [3][n]); moments [5][n], ics [6][n]."""
    _check(load().jeans_ics(C.byref(pot), _ptr(pos), _ptr(eps), pos.shape[1], float(h_R), float(h_z), float(b),
                            _ptr(moments), _ptr(ics), _stream()))


def dither_ics(ics, vc, u, dx, fv, out):
    """n_dither = u.shape[0] realisations of each initial condition into out [6][n*n_dither]."""
    _check(load().dither_ics(_ptr(ics), _ptr(vc), _ptr(u), ics.shape[1], u.shape[0], float(dx), float(fv), _ptr(out),
                             _stream()))


def bundle_rows(A, n_dither, out):
    """out[b] = mean of rows b*n_dither .. (b+1)*n_dither - 1 of A."""
    _check(load().bundle_rows(_ptr(A), _dtype_code(A), out.shape[0], A.shape[1], int(n_dither), _ptr(out), _stream()))


def integrate_bs23_workspace_bytes(n_orb, n_steps):
    return load().integrate_bs23_workspace_bytes(int(n_orb), int(n_steps))


def integrate_bs23_and_bin(pot, ics, h0, n_steps, rtol, atol, obs, A, overflow, drift, flags, workspace,
                           precision=SW_F64):
    """Adaptive BS23 orbits with time-weighted binning (FP64 tensors; the
    integration in `precision`, SW_F64 or SW_F32)."""
    _check(load().integrate_bs23_and_bin(C.byref(pot), _ptr(ics), _ptr(h0), ics.shape[1], int(n_steps), float(rtol),
                                         float(atol), int(precision), C.byref(obs), _ptr(A), _ptr(overflow),
                                         _ptr(drift), _ptr(flags), _ptr(workspace),
                                         workspace.numel() * workspace.element_size(), _stream()))


def integrate_orbits(pot, ics, dt, n_steps, out):
    _check(load().integrate_orbits(C.byref(pot), _ptr(ics), _ptr(dt), ics.shape[1], int(n_steps),
                                   _dtype_code(ics), _ptr(out), _stream()))


def mlp_param_count():
    return load().mlp_param_count()


def mlp_workspace_bytes(batch):
    return load().mlp_workspace_bytes(batch)


def mlp_forward(params, x, y, workspace):
    _check(load().mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(y), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream()))


def mlp_backward(params, x, dy, grad, workspace):
    _check(load().mlp_backward(_ptr(params), _ptr(x), x.shape[0], _ptr(dy), _ptr(grad), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream()))


def mlp_adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(t), lr, beta1, beta2,
                                eps, _stream()))


def mlp_pack_bf16(params, packed):
    _check(load().mlp_pack_bf16(_ptr(params), _ptr(packed), _stream()))


def mlp_infer_bf16(packed, x, y):
    _check(load().mlp_infer_bf16(_ptr(packed), _ptr(x), x.shape[0], _ptr(y), _stream()))


def mlp_mse_grad(y, t, dy):
    _check(load().mlp_mse_grad(_ptr(y), _ptr(t), y.shape[0], _ptr(dy), _stream()))


def set_tuning(key, value):
    _check(load().sw_set_tuning(key.encode(), int(value)))


def get_tuning(key):
    return load().sw_get_tuning(key.encode())
