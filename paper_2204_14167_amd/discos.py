"""ctypes binding of libdiscos.so (the C ABI in include/discos.h).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are torch tensors on the GPU (float64 / int32, contiguous); the stream is
torch's current HIP stream.  Importing this module does not load the library;
the first call does, and raises if the built library is missing.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiscos.so")

OK = 0
E_ARG, E_SHAPE, E_HIP, E_OUT_OF_DOMAIN, E_NOT_NEUTRAL, E_NONFINITE, E_CAPACITY = (
    -1, -2, -3, -4, -5, -6, -7)
E_NOT_CONVERGED = -8
BC_DIRICHLET, BC_NEUMANN = 0, 1
SPREAD_CHARGE, SPREAD_FORCE, SPREAD_ADD_BC = 0, 1, 0x100
INTERP_E, INTERP_FORCE, INTERP_PHI, INTERP_VEL = 0, 1, 2, 3
STEP_DRY, STEP_WET, STEP_RFD = 0, 1, 0x10
CREATE_HYDRO = 1
CREATE_MIXED_ITERATIVE = 2
CREATE_SERIAL = 4
MIXED_DENSE_MAX = 16384
STOKES_NOISE = 1
HYDRO_NOSLIP, HYDRO_SLIP = 0, 1
ADJ_REUSE_CELLS = 1

_c_dp = ctypes.POINTER(ctypes.c_double)


class DiscosGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double)]


class DiscosParams(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("bc_type", ctypes.c_int32 * 2),
        ("bc_value", ctypes.c_void_p * 2),
        ("e_ext", ctypes.c_double * 3),
        ("psi", ctypes.c_double),
        ("p3m_table", ctypes.c_void_p),
        ("p3m_len", ctypes.c_int32),
        ("p3m_dr", ctypes.c_double),
        ("wall_on", ctypes.c_int32),
        ("wall_sigma", ctypes.c_double),
        ("wall_xi", ctypes.c_double),
        ("wall_cut", ctypes.c_double),
        ("lj_on", ctypes.c_int32),
        ("lj_sigma", ctypes.c_void_p),
        ("lj_xi", ctypes.c_void_p),
        ("lj_cut_factor", ctypes.c_double),
        ("lj_range", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nspecies", ctypes.c_int32),
        ("radius", ctypes.c_void_p),
        ("mob_coef", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("rfd_delta", ctypes.c_double),
        ("hydro_bc", ctypes.c_int32 * 2),
        ("bc_type_map", ctypes.c_void_p * 2),
    ]


class DiscosIons(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("id", ctypes.c_void_p), ("species", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libdiscos.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2204_14167_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64
        L.discos_create.argtypes = [ctypes.POINTER(DiscosGrid), i64, ctypes.c_uint32,
                                    ctypes.POINTER(vp)]
        L.discos_destroy.argtypes = [vp]
        L.discos_spread.argtypes = [vp, i32, i64, vp, vp, ctypes.POINTER(DiscosParams), vp, vp]
        L.discos_solve_poisson.argtypes = [vp, vp, ctypes.POINTER(DiscosParams), vp, vp]
        L.discos_solve_stokes.argtypes = [vp, vp, ctypes.POINTER(DiscosParams), u64, i32, vp, vp,
                                          vp]
        L.discos_interpolate.argtypes = [vp, i32, i64, vp, vp, vp, ctypes.POINTER(DiscosParams),
                                         vp, vp]
        L.discos_near_field.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(DiscosParams), vp, vp]
        L.discos_step.argtypes = [vp, ctypes.POINTER(DiscosIons), ctypes.POINTER(DiscosParams),
                                  u64, i32, vp]
        L.discos_set_hydro_kernel.argtypes = [vp, i32, vp]
        L.discos_spread_force_species.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(DiscosParams),
                                                  vp, vp]
        L.discos_interpolate_vel_species.argtypes = [vp, i64, vp, vp, vp,
                                                     ctypes.POINTER(DiscosParams), vp, vp]
        L.discos_spread_charge_noalloc.argtypes = [ctypes.POINTER(DiscosGrid), i64, vp, vp,
                                                   ctypes.POINTER(DiscosParams), ctypes.c_uint32,
                                                   vp, vp, vp]
        L.discos_check.argtypes = [vp]
        L.discos_profile.argtypes = [vp, i32]
        L.discos_profile_stages.argtypes = [vp, ctypes.c_uint32]
        L.discos_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int)]
        L.discos_energy_flux.argtypes = [vp, i64, vp, vp, ctypes.POINTER(DiscosParams), vp, vp, vp]
        L.discos_energy_flux_backward.argtypes = [vp, i64, vp, vp, ctypes.POINTER(DiscosParams), vp, vp,
                                                  vp, vp, vp, vp, vp, ctypes.c_uint32, vp]
        L.discos_batch_create.argtypes = [ctypes.POINTER(DiscosReplica), i32, ctypes.c_double,
                                          ctypes.POINTER(DiscosParams), ctypes.POINTER(vp)]
        L.discos_batch_destroy.argtypes = [vp]
        L.discos_batch_step.argtypes = [vp, vp, vp, vp, vp, u64, ctypes.c_uint32, vp]
        L.discos_batch_tune.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
        L.discos_batch_set_bin.argtypes = [vp, i32]
        L.discos_batch_check.argtypes = [vp]
        L.discos_batch_last_error.argtypes = [vp]
        L.discos_batch_last_error.restype = ctypes.c_char_p
        L.discos_last_error.argtypes = [vp]
        L.discos_last_error.restype = ctypes.c_char_p
        for name in ("discos_create", "discos_destroy", "discos_spread", "discos_solve_poisson",
                     "discos_solve_stokes",
                     "discos_interpolate", "discos_near_field", "discos_step", "discos_check",
                     "discos_profile", "discos_profile_read", "discos_energy_flux",
                     "discos_energy_flux_backward", "discos_batch_create", "discos_batch_destroy",
                     "discos_batch_step", "discos_batch_tune", "discos_batch_set_bin", "discos_batch_check",
                     "discos_set_hydro_kernel", "discos_spread_force_species",
                     "discos_interpolate_vel_species", "discos_profile_stages",
                     "discos_spread_charge_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class DiscosReplica(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n", ctypes.c_int64), ("bc_value", ctypes.c_double * 2),
                ("seed", ctypes.c_uint64), ("mob_coef", ctypes.c_void_p)]


class DiscosError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"discos error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f64(a, device):
    return torch.as_tensor(np.array(a, dtype=np.float64, copy=True, order="C"), device=device)


class Params:
    """Device copy of a parameter dict (keys as produced by workloads.make_params)
    plus the ctypes struct pointing into it."""

    def __init__(self, p, grid, device="cuda"):
        nx, ny = grid[0], grid[1]
        self._keep = []
        s = DiscosParams()
        s.eps = p["eps"]
        for w in (0, 1):
            t = p["bc_types"][w]
            if np.ndim(t) == 0:
                s.bc_type[w] = int(t)
                s.bc_type_map[w] = None
            else:
                # a wall of mixed type: the type of every column (the library reads it)
                m = torch.as_tensor(np.array(np.broadcast_to(t, (ny, nx)), dtype=np.int32, copy=True),
                                    device=device)
                self._keep.append(m)
                s.bc_type_map[w] = m.data_ptr()
                s.bc_type[w] = BC_DIRICHLET if bool(np.any(np.asarray(t) == BC_DIRICHLET)) else BC_NEUMANN
        for w in (0, 1):
            v = p["bc_values"][w] if p.get("bc_values") is not None else None
            if v is None:
                s.bc_value[w] = None
            elif isinstance(v, torch.Tensor) and v.device.type == "cuda":
                # used in place (the autograd path): must be float64 [ny][nx], contiguous
                if v.dtype != torch.float64 or tuple(v.shape) != (ny, nx) or not v.is_contiguous():
                    raise ValueError("wall field tensors must be contiguous float64 [ny, nx]")
                self._keep.append(v)
                s.bc_value[w] = v.data_ptr()
            else:
                t = _f64(np.broadcast_to(np.asarray(v, dtype=np.float64), (ny, nx)), device)
                self._keep.append(t)
                s.bc_value[w] = t.data_ptr()
        e = p.get("e_ext", (0.0, 0.0, 0.0))
        for k in range(3):
            s.e_ext[k] = float(e[k])
        s.psi = p.get("psi", 4.0)
        if p.get("p3m_table") is not None:
            t = _f64(p["p3m_table"], device)
            self._keep.append(t)
            s.p3m_table = t.data_ptr()
            s.p3m_len = t.numel()
            s.p3m_dr = p["p3m_dr"]
        s.wall_on = int(bool(p.get("wall_on", False)))
        s.wall_sigma = p.get("wall_sigma", 1.0)
        s.wall_xi = p.get("wall_xi", 1.0)
        s.wall_cut = p.get("wall_cut", 3.5)
        s.lj_on = int(bool(p.get("lj_on", False)))
        if s.lj_on:
            ls = _f64(p["lj_sigma"], device)
            lx = _f64(p["lj_xi"], device)
            self._keep += [ls, lx]
            s.lj_sigma, s.lj_xi = ls.data_ptr(), lx.data_ptr()
            s.lj_cut_factor = p["lj_cut_factor"]
            s.lj_range = float(p["lj_cut_factor"] * np.max(p["lj_sigma"]))
        s.kT = p.get("kT", 1.0)
        s.eta = p.get("eta", 1.0)
        s.dt = p.get("dt", 0.0)
        if p.get("radius") is not None:
            r = _f64(p["radius"], device)
            self._keep.append(r)
            s.radius = r.data_ptr()
            s.nspecies = r.numel()
        if p.get("mob_coef") is not None:
            c = _f64(p["mob_coef"], device)
            self._keep.append(c)
            s.mob_coef = c.data_ptr()
        s.seed = int(p.get("seed", 0))
        s.rfd_delta = float(p.get("rfd_delta", 0.0))
        # hydrodynamic walls: p["slip"] = (lower, upper), default no-slip
        sl = p.get("slip", (False, False))
        s.hydro_bc[0] = HYDRO_SLIP if sl[0] else HYDRO_NOSLIP
        s.hydro_bc[1] = HYDRO_SLIP if sl[1] else HYDRO_NOSLIP
        self.struct = s


NOALLOC_MAX_IONS, NOALLOC_MAX_BINS = 65536, 262144


def spread_charge_noalloc(grid, pos, q, params, add_bc=False, out=None, status=None):
    """rho = S^es q through discos_spread_charge_noalloc (no context, no allocation in the
    library).  grid = (nx, ny, nz, h); params from Params(p, grid); out [nz, ny, nx] and
    status (int32 [1], receives the call's device condition) are optional device tensors."""
    nx, ny, nz, h = grid
    g = DiscosGrid(int(nx), int(ny), int(nz), float(h))
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float64, device=pos.device)
    rc = lib().discos_spread_charge_noalloc(ctypes.byref(g), pos.shape[1], _ptr(pos), _ptr(q),
                                            ctypes.byref(params.struct),
                                            SPREAD_ADD_BC if add_bc else 0, _ptr(out),
                                            _ptr(status), _stream())
    if rc != OK:
        raise DiscosError(rc, "discos_spread_charge_noalloc failed")
    return out


class Context:
    """One grid and up to n_max ions; owns the library context."""

    def __init__(self, nx, ny, nz, h=1.0, n_max=0, hydro=False, mixed_iterative=False,
                 serial=False):
        """mixed_iterative: walls of mixed type by conjugate gradients only (no dense
        inverse of their capacitance system).  serial: every stage of a step in order on
        the caller's stream (no second stream for the dry step's near field)."""
        self.grid = (int(nx), int(ny), int(nz), float(h))
        g = DiscosGrid(int(nx), int(ny), int(nz), float(h))
        h_ = ctypes.c_void_p()
        flags = ((CREATE_HYDRO if hydro else 0) | (CREATE_MIXED_ITERATIVE if mixed_iterative else 0)
                 | (CREATE_SERIAL if serial else 0))
        rc = lib().discos_create(ctypes.byref(g), int(n_max), flags, ctypes.byref(h_))
        if rc != OK:
            raise DiscosError(rc, "discos_create failed")
        self.handle = h_
        self.n_max = int(n_max)

    def close(self):
        """Release the context (waits for the device).  Raises DiscosError if the runtime
        reported an error on the way; the context is released regardless."""
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            rc = lib().discos_destroy(h)
            if rc != OK:
                raise DiscosError(rc, "device error while releasing the context")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc):
        if rc != OK:
            raise DiscosError(rc, lib().discos_last_error(self.handle).decode())

    def params(self, p, device="cuda"):
        return Params(p, self.grid, device)

    @property
    def cell_shape(self):
        nx, ny, nz, _ = self.grid
        return (nz, ny, nx)

    # ---- entry points (same names as the C ABI) ---------------------------------
    @property
    def face_size(self):
        nx, ny, nz, _ = self.grid
        return 2 * nx * ny * nz + nx * ny * (nz + 1)

    def split_faces(self, a):
        """(u, v, w) views of a flat face array."""
        nx, ny, nz, _ = self.grid
        c = nx * ny * nz
        return (a[:c].view(nz, ny, nx), a[c:2 * c].view(nz, ny, nx),
                a[2 * c:].view(nz + 1, ny, nx))

    def spread(self, op, pos, w, params, out=None):
        nz, ny, nx = self.cell_shape
        if out is None:
            shape = (self.face_size,) if (op & 0xFF) == SPREAD_FORCE else (nz, ny, nx)
            out = torch.empty(shape, dtype=torch.float64, device=pos.device)
        self._rc(lib().discos_spread(self.handle, op, pos.shape[1], _ptr(pos), _ptr(w),
                                     ctypes.byref(params.struct), _ptr(out), _stream()))
        return out

    def solve_poisson(self, rhs, params, out=None):
        if out is None:
            out = torch.empty_like(rhs)
        self._rc(lib().discos_solve_poisson(self.handle, _ptr(rhs), ctypes.byref(params.struct),
                                            _ptr(out), _stream()))
        return out

    def solve_stokes(self, f, params, step=0, noise=False, out=None, pres=None):
        if out is None:
            out = torch.empty_like(f)
        self._rc(lib().discos_solve_stokes(self.handle, _ptr(f), ctypes.byref(params.struct),
                                           int(step), STOKES_NOISE if noise else 0, _ptr(out),
                                           _ptr(pres), _stream()))
        return out

    def interpolate(self, op, pos, field, params, aux=None, out=None):
        n = pos.shape[1]
        if out is None:
            shape = (n,) if op == INTERP_PHI else (3, n)
            out = torch.empty(shape, dtype=torch.float64, device=pos.device)
        self._rc(lib().discos_interpolate(self.handle, op, n, _ptr(pos), _ptr(field), _ptr(aux),
                                          ctypes.byref(params.struct), _ptr(out), _stream()))
        return out

    def set_hydro_kernel(self, kernels):
        """Hydrodynamic kernel per species: a sequence of (w, beta), w = 0 for the 4-point
        Peskin kernel, w = 2 .. 8 for the ESC kernel of App. B; None or [] restores Peskin."""
        rows = [] if kernels is None else [(float(w), float(b)) for w, b in kernels]
        buf = (ctypes.c_double * max(2 * len(rows), 1))(*[v for r in rows for v in r])
        self._rc(lib().discos_set_hydro_kernel(self.handle, len(rows),
                                               ctypes.cast(buf, ctypes.c_void_p)))

    def spread_species(self, pos, F, species, params, out=None):
        """S^hy F with each ion's kernel chosen by its species (int32, device)."""
        if out is None:
            out = torch.empty((self.face_size,), dtype=torch.float64, device=pos.device)
        self._rc(lib().discos_spread_force_species(self.handle, pos.shape[1], _ptr(pos), _ptr(F),
                                                   _ptr(species), ctypes.byref(params.struct),
                                                   _ptr(out), _stream()))
        return out

    def interpolate_vel_species(self, pos, v, species, params, out=None):
        """J^hy v with each ion's kernel chosen by its species (int32, device)."""
        n = pos.shape[1]
        if out is None:
            out = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        self._rc(lib().discos_interpolate_vel_species(self.handle, n, _ptr(pos), _ptr(v),
                                                      _ptr(species), ctypes.byref(params.struct),
                                                      _ptr(out), _stream()))
        return out

    def near_field(self, pos, q, params, species=None, F=None):
        n = pos.shape[1]
        if F is None:
            F = torch.zeros((3, n), dtype=torch.float64, device=pos.device)
        self._rc(lib().discos_near_field(self.handle, n, _ptr(pos), _ptr(q), _ptr(species),
                                         ctypes.byref(params.struct), _ptr(F), _stream()))
        return F

    def step(self, pos, q, ids, species, params, step, mode=STEP_DRY):
        ions = DiscosIons(pos.shape[1], pos.data_ptr(), q.data_ptr(), ids.data_ptr(),
                          species.data_ptr())
        self._rc(lib().discos_step(self.handle, ctypes.byref(ions), ctypes.byref(params.struct),
                                   int(step), mode, _stream()))

    STAGES = ("cell_list", "spread", "fft_x", "fft_y", "z_solve", "ifft_y", "ifft_x",
              "interp", "near_list", "near_field", "spread_hy", "stokes", "interp_hy", "update")

    def profile(self, enable=True):
        self._rc(lib().discos_profile(self.handle, int(enable)))

    def profile_stages(self, names):
        """Time only the named stages (their two bounding events per step); [] stops."""
        mask = 0
        for nm in names:
            mask |= 1 << self.STAGES.index(nm)
        self._rc(lib().discos_profile_stages(self.handle, mask))

    def profile_read(self):
        """{stage: ms}, the mean over the steps profiled since profiling was enabled
        (synchronises)."""
        ms = (ctypes.c_double * 16)()
        cnt = ctypes.c_int()
        self._rc(lib().discos_profile_read(self.handle, ms, ctypes.byref(cnt)))
        return {self.STAGES[k]: ms[k] for k in range(cnt.value)}

    def energy_flux(self, pos, q, params, phi=None, out=None):
        """(out, phi): out = [U, Q] (device), phi the checkpoint of the backward pass."""
        n = pos.shape[1] if pos is not None else 0
        nx, ny, nz, _ = self.grid
        if phi is None:
            phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device="cuda")
        self._rc(lib().discos_energy_flux(self.handle, n, _ptr(pos), _ptr(q), ctypes.byref(params.struct),
                                          _ptr(phi), _ptr(out), _stream()))
        return out, phi

    def energy_flux_backward(self, pos, q, params, phi, g, want=("pos", "q", "bc_lo", "bc_hi", "e_ext"),
                             reuse_cells=False):
        """gU dU + gQ dQ (g = [gU, gQ] on the device) w.r.t. the requested inputs.
        reuse_cells: pos and q are unchanged since the energy_flux call that wrote phi, so
        its cell list may serve again (the library rebuilds it if another call did)."""
        n = pos.shape[1] if pos is not None else 0
        nx, ny, nz, _ = self.grid
        dev = dict(dtype=torch.float64, device="cuda")
        res = {}
        res["pos"] = torch.empty((3, n), **dev) if "pos" in want else None
        res["q"] = torch.empty(n, **dev) if "q" in want else None
        res["bc_lo"] = torch.empty((ny, nx), **dev) if "bc_lo" in want else None
        res["bc_hi"] = torch.empty((ny, nx), **dev) if "bc_hi" in want else None
        res["e_ext"] = torch.empty(3, **dev) if "e_ext" in want else None
        self._rc(lib().discos_energy_flux_backward(
            self.handle, n, _ptr(pos), _ptr(q), ctypes.byref(params.struct), _ptr(phi), _ptr(g),
            _ptr(res["pos"]), _ptr(res["q"]), _ptr(res["bc_lo"]), _ptr(res["bc_hi"]), _ptr(res["e_ext"]),
            ADJ_REUSE_CELLS if reuse_cells else 0, _stream()))
        return res

    def check(self):
        """Synchronise and raise on a sticky device-side error."""
        self._rc(lib().discos_check(self.handle))


BATCH_GRAPH = 1


class Batch:
    """A batch of independent channels (library discos_batch).  `reps` is a list of
    dicts with nx, ny, nz, n, bc_values (two scalars), seed and optionally mob_coef
    (a [nspecies, 2, 7] array); `params` the shared physics (keys of make_params)."""

    def __init__(self, reps, h, params, device="cuda"):
        self._keep = []
        p = dict(params)
        p["bc_values"] = (None, None)
        self.params = Params(p, (reps[0]["nx"], reps[0]["ny"]), device)
        arr = (DiscosReplica * len(reps))()
        coefs = {}
        for k, r in enumerate(reps):
            arr[k].nx, arr[k].ny, arr[k].nz = int(r["nx"]), int(r["ny"]), int(r["nz"])
            arr[k].n = int(r["n"])
            arr[k].bc_value[0] = float(r["bc_values"][0])
            arr[k].bc_value[1] = float(r["bc_values"][1])
            arr[k].seed = int(r["seed"])
            c = r.get("mob_coef")
            if c is not None:
                key = np.asarray(c, dtype=np.float64).tobytes()
                if key not in coefs:
                    coefs[key] = _f64(c, device)
                arr[k].mob_coef = coefs[key].data_ptr()
        self._keep += list(coefs.values())
        self.offsets = np.concatenate([[0], np.cumsum([int(r["n"]) for r in reps])])
        h_ = ctypes.c_void_p()
        rc = lib().discos_batch_create(arr, len(reps), float(h), ctypes.byref(self.params.struct),
                                       ctypes.byref(h_))
        if rc != OK:
            raise DiscosError(rc, "discos_batch_create failed")
        self.handle = h_

    def close(self):
        """Release the batch (waits for the device); raises as Context.close does."""
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            rc = lib().discos_batch_destroy(h)
            if rc != OK:
                raise DiscosError(rc, "device error while releasing the batch")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc):
        if rc != OK:
            raise DiscosError(rc, lib().discos_batch_last_error(self.handle).decode())

    def step(self, pos, q, ids, species, step, graph=False):
        self._rc(lib().discos_batch_step(self.handle, _ptr(pos), _ptr(q), _ptr(ids), _ptr(species),
                                         int(step), BATCH_GRAPH if graph else 0, _stream()))

    def tune(self, pos, q, ids, species):
        cfg = (ctypes.c_int32 * 10)()
        self._rc(lib().discos_batch_tune(self.handle, _ptr(pos), _ptr(q), _ptr(ids), _ptr(species),
                                         cfg, _stream()))
        return dict(spread_tile=cfg[0], spread_blocks=cfg[1], interp_tile=cfg[2],
                    interp_blocks=cfg[3], ion_block=cfg[4], interp_direct=cfg[5],
                    spread_direct=cfg[6], bin=cfg[7], bin_us={2: cfg[8], 4: cfg[9]})

    def set_bin(self, bin_cells):
        """Cell-list bin edge in cells (2 or 4), as the autotuner chooses it."""
        self._rc(lib().discos_batch_set_bin(self.handle, int(bin_cells)))

    def check(self):
        self._rc(lib().discos_batch_check(self.handle))

