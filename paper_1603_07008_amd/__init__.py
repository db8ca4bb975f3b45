"""MI355X-native mixed-precision sLdG projection sweep (arXiv 1603.07008).

Thin ctypes binding of libsldg.so (C ABI in include/sldg.h).  The functions
here only marshal arguments (device pointers of torch tensors, the current HIP
stream) and check buffer sizes; every step of the sweep runs in the library's
HIP kernels.  There is no CPU fallback: without the built library every call
raises.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsldg.so")

SLDG_OK, SLDG_ERR_ARG, SLDG_ERR_ALIAS, SLDG_ERR_UNSUPPORTED, SLDG_ERR_NOMEM, SLDG_ERR_DEVICE = range(6)
TIERS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
TIER_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}
SLDG_SHAPE_STAGED = 16    # colwaves flag: strided tile staged through LDS
SLDG_SHAPE_MEMORDER = 32  # colwaves flag: strided tiles in memory order
SWEEP_FORMS = ("window", "group", "strided", "lane", "staged")

EXPORTS = ("sldg_plan", "sldg_plan_destroy", "sldg_plan_set_stream", "sldg_line_tables",
           "sldg_advect_dim", "sldg_split_steps", "sldg_mass", "sldg_hi_bytes",
           "sldg_status_string", "sldg_last_error", "sldg_timing_enable", "sldg_timing_read",
           "sldg_mass_device", "sldg_device_copy", "sldg_advect_dim_adjoint",
           "sldg_batch_create", "sldg_batch_destroy", "sldg_batch_bind", "sldg_batch_set_sequence",
           "sldg_batch_run", "sldg_batch_tune", "sldg_batch_get_tuning", "sldg_batch_set_tuning",
           "sldg_plan_ex", "sldg_lo_planes", "sldg_hi_planes", "sldg_plane_map",
           "sldg_scale_bytes", "sldg_set_scale_headroom", "sldg_scaled_import",
           "sldg_scaled_export", "sldg_advect_dim_scaled", "sldg_split_steps_scaled",
           "sldg_plan_set_shape", "sldg_plan_get_shape", "sldg_plan_sweep_form",
           "sldg_tune_candidate", "sldg_plan_tune",
           "sldg_device_plane_copy", "sldg_batch_get_class_tuning", "sldg_batch_set_class_tuning",
           "sldg_poisson_shift", "sldg_poisson_shift_noalloc", "sldg_vlasov_poisson_steps",
           "sldg_advect_dim_collocated", "sldg_poisson_shift_2d", "sldg_vlasov_poisson_steps_2d2v",
           "sldg_set_device_alloc_limit", "sldg_device_alloc_bytes", "sldg_advect_dims01",
           "sldg_plan_set_fusion")


class SldgError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({detail})")


class SweepDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("dep_mask", ctypes.c_uint32), ("shift", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libsldg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsldg.so is not built ({LIB_PATH}); run paper_1603_07008_amd/build.py")
    # torch's HIP runtime is loaded first, so that the library binds to the
    # same runtime (same soname) as the tensors whose pointers it is given
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
    L.sldg_plan.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i64), i32, i32, vp]
    L.sldg_plan.restype = i32
    L.sldg_plan_ex.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i64), i32, i32, i32, vp]
    L.sldg_plan_ex.restype = i32
    L.sldg_lo_planes.argtypes = [vp]
    L.sldg_lo_planes.restype = i64
    L.sldg_hi_planes.argtypes = [vp]
    L.sldg_hi_planes.restype = i64
    L.sldg_plane_map.argtypes = [vp, vp]
    L.sldg_plane_map.restype = i32
    L.sldg_plan_destroy.argtypes = [vp]
    L.sldg_plan_destroy.restype = None
    L.sldg_plan_set_stream.argtypes = [vp, vp]
    L.sldg_plan_set_stream.restype = i32
    L.sldg_line_tables.argtypes = [vp, i64, i64, vp, vp, vp]
    L.sldg_line_tables.restype = i32
    L.sldg_advect_dim.argtypes = [vp, i32, vp, u32, vp, vp, vp, vp]
    L.sldg_advect_dim.restype = i32
    L.sldg_advect_dim_adjoint.argtypes = [vp, i32, vp, u32, vp, vp, vp, vp]
    L.sldg_advect_dim_adjoint.restype = i32
    L.sldg_split_steps.argtypes = [vp, ctypes.POINTER(SweepDesc), i32, i32, vp, vp, vp, vp,
                                   ctypes.POINTER(i32)]
    L.sldg_split_steps.restype = i32
    L.sldg_mass.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.sldg_mass.restype = i32
    L.sldg_hi_bytes.argtypes = [vp]
    L.sldg_hi_bytes.restype = i64
    L.sldg_device_copy.argtypes = [vp, vp, i64, vp]
    L.sldg_device_copy.restype = i32
    L.sldg_device_plane_copy.argtypes = [vp, vp, i64, i32, i32, vp]
    L.sldg_device_plane_copy.restype = i32
    L.sldg_mass_device.argtypes = [vp, vp, vp]
    L.sldg_mass_device.restype = i32
    L.sldg_timing_enable.argtypes = [vp, i32]
    L.sldg_timing_enable.restype = i32
    L.sldg_timing_read.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.sldg_timing_read.restype = i32
    L.sldg_scale_bytes.argtypes = [vp]
    L.sldg_scale_bytes.restype = i64
    L.sldg_set_scale_headroom.argtypes = [vp, i32]
    L.sldg_set_scale_headroom.restype = i32
    L.sldg_scaled_import.argtypes = [vp, vp, vp, vp]
    L.sldg_scaled_import.restype = i32
    L.sldg_scaled_export.argtypes = [vp, vp, vp, vp]
    L.sldg_scaled_export.restype = i32
    L.sldg_advect_dim_scaled.argtypes = [vp, i32, vp, u32, vp, vp, vp, vp, vp, vp]
    L.sldg_advect_dim_scaled.restype = i32
    L.sldg_split_steps_scaled.argtypes = [vp, ctypes.POINTER(SweepDesc), i32, i32, vp, vp, vp,
                                          vp, vp, vp, ctypes.POINTER(i32)]
    L.sldg_split_steps_scaled.restype = i32
    L.sldg_plan_set_shape.argtypes = [vp, i32, i32, i32, i32]
    L.sldg_plan_set_shape.restype = i32
    L.sldg_plan_get_shape.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
    L.sldg_plan_get_shape.restype = i32
    L.sldg_plan_sweep_form.argtypes = [vp, i32, ctypes.c_uint32, vp, vp, vp, vp,
                                       ctypes.POINTER(i32)]
    L.sldg_plan_sweep_form.restype = i32
    L.sldg_tune_candidate.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
    L.sldg_tune_candidate.restype = i32
    L.sldg_plan_tune.argtypes = [vp, ctypes.POINTER(SweepDesc), i32, vp, vp, vp, vp, i32,
                                 ctypes.POINTER(ctypes.c_double)]
    L.sldg_plan_tune.restype = i32
    dbl = ctypes.c_double
    L.sldg_advect_dim_collocated.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.sldg_advect_dim_collocated.restype = i32
    L.sldg_poisson_shift.argtypes = [vp, vp, vp, dbl, dbl, dbl, vp, vp]
    L.sldg_poisson_shift.restype = i32
    L.sldg_poisson_shift_noalloc.argtypes = [vp, vp, vp, dbl, dbl, dbl, vp, vp]
    L.sldg_poisson_shift_noalloc.restype = i32
    L.sldg_vlasov_poisson_steps.argtypes = [vp, i32, vp, dbl, dbl, dbl, vp, vp, vp, vp, vp,
                                            ctypes.POINTER(i32)]
    L.sldg_vlasov_poisson_steps.restype = i32
    L.sldg_poisson_shift_2d.argtypes = [vp, vp, vp, ctypes.POINTER(dbl), dbl, vp, vp, vp]
    L.sldg_poisson_shift_2d.restype = i32
    L.sldg_vlasov_poisson_steps_2d2v.argtypes = [vp, i32, vp, vp, ctypes.POINTER(dbl), dbl, vp,
                                                 vp, vp, vp, vp, vp, ctypes.POINTER(i32)]
    L.sldg_vlasov_poisson_steps_2d2v.restype = i32
    L.sldg_advect_dims01.argtypes = [vp, vp, u32, vp, u32, vp, vp, vp, vp]
    L.sldg_advect_dims01.restype = i32
    L.sldg_plan_set_fusion.argtypes = [vp, i32]
    L.sldg_plan_set_fusion.restype = i32
    L.sldg_set_device_alloc_limit.argtypes = [i64]
    L.sldg_set_device_alloc_limit.restype = i32
    L.sldg_device_alloc_bytes.argtypes = []
    L.sldg_device_alloc_bytes.restype = i64
    L.sldg_status_string.argtypes = [i32]
    L.sldg_status_string.restype = ctypes.c_char_p
    L.sldg_last_error.argtypes = []
    L.sldg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status):
    return lib().sldg_status_string(int(status)).decode()


def last_error():
    return lib().sldg_last_error().decode()


def _check(status, where):
    if status != SLDG_OK:
        raise SldgError(status, where, last_error())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def hi_dtype(tier):
    import torch
    return {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16,
            "fp16": torch.float16}[tier]


class Plan:
    """A grid + degree + storage tier (sldg_plan).  Calls are enqueued on the
    HIP stream given at creation (default: torch's current stream)."""

    def __init__(self, ncells, k, tier="fp32", stream=None, ndouble=1):
        self.ncells = tuple(int(n) for n in ncells)
        self.ndim = len(self.ncells)
        self.k = int(k)
        self.tier = tier
        self.cells = 1
        for n in self.ncells:
            self.cells *= n
        self.modes = (self.k + 1) ** self.ndim
        if tier not in TIERS:
            raise ValueError(f"unknown tier {tier!r}")
        self.stream = _current_stream() if stream is None else stream
        self.ndouble = int(ndouble)
        h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * self.ndim)(*self.ncells)
        _check(lib().sldg_plan_ex(ctypes.byref(h), self.ndim, arr, self.k, TIERS[tier],
                                  self.ndouble, ctypes.c_void_p(self.stream)), "sldg_plan_ex")
        self._h = h
        self.n_lo = int(lib().sldg_lo_planes(h))
        self.n_hi = int(lib().sldg_hi_planes(h))

    # -- helpers -----------------------------------------------------------
    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def hi_bytes(self):
        return int(lib().sldg_hi_bytes(self.handle))

    def plane_map(self):
        """Per mode id: >= 0 plane of `hi`, < 0 plane -1-v of `mass` (sldg_plane_map)."""
        out = (ctypes.c_int32 * self.modes)()
        _check(lib().sldg_plane_map(self.handle, out), "sldg_plane_map")
        return list(out)

    def empty_state(self, device="cuda"):
        """Uninitialised (mass, hi) device tensors of this plan's layout: mass is
        [cells] when it holds mode 0 alone, else [n_lo, cells]."""
        import torch
        shape = (self.cells,) if self.n_lo == 1 else (self.n_lo, self.cells)
        mass = torch.empty(shape, dtype=torch.float64, device=device)
        hi = torch.empty((self.n_hi, self.cells), dtype=hi_dtype(self.tier), device=device)
        return mass, hi

    def _check_state(self, mass, hi, what):
        import torch
        if not isinstance(mass, torch.Tensor) or not isinstance(hi, torch.Tensor):
            raise TypeError(f"{what}: state buffers must be torch tensors")
        if not (mass.is_cuda and hi.is_cuda):
            raise ValueError(f"{what}: state buffers must be device tensors")
        if mass.dtype != torch.float64 or not mass.is_contiguous() or \
                mass.numel() < self.n_lo * self.cells:
            raise ValueError(f"{what}: mass must be contiguous float64 with >= "
                             f"{self.n_lo * self.cells} elements")
        if hi.dtype != hi_dtype(self.tier) or not hi.is_contiguous() or \
                hi.numel() * hi.element_size() < self.hi_bytes():
            raise ValueError(f"{what}: hi must be contiguous {hi_dtype(self.tier)} of "
                             f"{self.hi_bytes()} bytes")

    def _check_shift(self, shift, dep_mask, what):
        import torch
        need = 1
        for e in range(self.ndim):
            if dep_mask >> e & 1:
                need *= self.ncells[e]
        if not isinstance(shift, torch.Tensor) or not shift.is_cuda or \
                shift.dtype != torch.float64 or not shift.is_contiguous() or shift.numel() < need:
            raise ValueError(f"{what}: shift must be a contiguous float64 device tensor of "
                             f">= {need} elements")

    # -- C entry points ----------------------------------------------------
    def set_stream(self, stream):
        self.stream = stream
        _check(lib().sldg_plan_set_stream(self.handle, ctypes.c_void_p(stream)), "sldg_plan_set_stream")

    def line_tables(self, sigma, period, s_out=None, ab_out=None):
        """(s mod period, [A; B]) per displacement (sldg_line_tables)."""
        import torch
        n = sigma.numel()
        if sigma.dtype != torch.float64 or not sigma.is_cuda or not sigma.is_contiguous():
            raise ValueError("sigma must be a contiguous float64 device tensor")
        o = self.k + 1
        if s_out is None:
            s_out = torch.empty(n, dtype=torch.int32, device=sigma.device)
        if ab_out is None:
            ab_out = torch.empty((n, 2, o, o), dtype=torch.float64, device=sigma.device)
        if s_out.numel() < n or ab_out.numel() < n * 2 * o * o:
            raise ValueError("output tables too small")
        _check(lib().sldg_line_tables(self.handle, n, int(period), _ptr(sigma), _ptr(s_out),
                                      _ptr(ab_out)), "sldg_line_tables")
        return s_out, ab_out

    def advect_dim(self, dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi):
        """One projection sweep along `dim` (sldg_advect_dim)."""
        self._check_shift(shift, dep_mask, "advect_dim")
        self._check_state(in_mass, in_hi, "advect_dim input")
        self._check_state(out_mass, out_hi, "advect_dim output")
        _check(lib().sldg_advect_dim(self.handle, int(dim), _ptr(shift), int(dep_mask),
                                     _ptr(in_mass), _ptr(in_hi), _ptr(out_mass), _ptr(out_hi)),
               "sldg_advect_dim")

    def advect_dims01(self, shift0, dep_mask0, shift1, dep_mask1, in_mass, in_hi, out_mass,
                      out_hi):
        """The sweep along dimension 0 then the sweep along dimension 1 in one
        fused pass (sldg_advect_dims01); bitwise two advect_dim calls."""
        self._check_shift(shift0, dep_mask0, "advect_dims01")
        self._check_shift(shift1, dep_mask1, "advect_dims01")
        self._check_state(in_mass, in_hi, "advect_dims01 input")
        self._check_state(out_mass, out_hi, "advect_dims01 output")
        _check(lib().sldg_advect_dims01(self.handle, _ptr(shift0), int(dep_mask0), _ptr(shift1),
                                        int(dep_mask1), _ptr(in_mass), _ptr(in_hi),
                                        _ptr(out_mass), _ptr(out_hi)), "sldg_advect_dims01")

    def set_fusion(self, enable):
        """Fusion of (0, 1) sweep pairs in split_steps (sldg_plan_set_fusion)."""
        _check(lib().sldg_plan_set_fusion(self.handle, 1 if enable else 0), "sldg_plan_set_fusion")

    def advect_dim_adjoint(self, dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi):
        """The transposed sweep (sldg_advect_dim_adjoint)."""
        self._check_shift(shift, dep_mask, "advect_dim_adjoint")
        self._check_state(in_mass, in_hi, "advect_dim_adjoint input")
        self._check_state(out_mass, out_hi, "advect_dim_adjoint output")
        _check(lib().sldg_advect_dim_adjoint(self.handle, int(dim), _ptr(shift), int(dep_mask),
                                             _ptr(in_mass), _ptr(in_hi), _ptr(out_mass),
                                             _ptr(out_hi)), "sldg_advect_dim_adjoint")

    def split_steps(self, seq, nsteps, state0, state1):
        """Apply the sweeps `seq` [(dim, dep_mask, shift tensor), ...] nsteps
        times, ping-ponging between state0 and state1 (sldg_split_steps).
        Returns the index (0 or 1) of the state that holds the result."""
        descs = (SweepDesc * max(1, len(seq)))()
        for q, (dim, mask, shift) in enumerate(seq):
            self._check_shift(shift, mask, "split_steps")
            descs[q] = SweepDesc(int(dim), int(mask), _ptr(shift))
        self._check_state(*state0, "split_steps state0")
        self._check_state(*state1, "split_steps state1")
        res = ctypes.c_int(-1)
        _check(lib().sldg_split_steps(self.handle, descs, len(seq), int(nsteps),
                                      _ptr(state0[0]), _ptr(state0[1]), _ptr(state1[0]),
                                      _ptr(state1[1]), ctypes.byref(res)), "sldg_split_steps")
        return res.value

    def advect_dim_collocated(self, dim, tdim, node_shift, in_mass, in_hi, out_mass, out_hi):
        """Sweep along `dim` with Gauss-node collocation in `tdim`
        (sldg_advect_dim_collocated); node_shift: float64 device
        [N_tdim * (k+1)], node fastest."""
        import torch
        need = self.ncells[tdim] * (self.k + 1)
        if not isinstance(node_shift, torch.Tensor) or not node_shift.is_cuda or \
                node_shift.dtype != torch.float64 or not node_shift.is_contiguous() or \
                node_shift.numel() < need:
            raise ValueError(f"advect_dim_collocated: node_shift must be a contiguous float64 "
                             f"device tensor of >= {need} elements")
        self._check_state(in_mass, in_hi, "advect_dim_collocated input")
        self._check_state(out_mass, out_hi, "advect_dim_collocated output")
        _check(lib().sldg_advect_dim_collocated(self.handle, int(dim), int(tdim), _ptr(node_shift),
                                                _ptr(in_mass), _ptr(in_hi), _ptr(out_mass),
                                                _ptr(out_hi)), "sldg_advect_dim_collocated")

    # --- self-consistent field of (x, v) problems ---------------------------

    def poisson_shift(self, mass, hi, hx, hv, dt, shift_out=None, field_out=None):
        """The v-sweep displacements E(x_i) dt / hv of the state's field
        (sldg_poisson_shift); returns shift_out (device float64 [N_x])."""
        return self._poisson_shift("sldg_poisson_shift", mass, hi, hx, hv, dt, shift_out,
                                   field_out)

    def poisson_shift_noalloc(self, mass, hi, hx, hv, dt, shift_out=None, field_out=None):
        """poisson_shift through the allocation-free entry point
        (sldg_poisson_shift_noalloc: static device scratch; calls that overlap
        on one device race)."""
        return self._poisson_shift("sldg_poisson_shift_noalloc", mass, hi, hx, hv, dt, shift_out,
                                   field_out)

    def _poisson_shift(self, entry, mass, hi, hx, hv, dt, shift_out, field_out):
        import torch
        self._check_state(mass, hi, "poisson_shift")
        nx = self.ncells[0]
        if shift_out is None:
            shift_out = torch.empty(nx, dtype=torch.float64, device=mass.device)
        for t, nm in ((shift_out, "shift_out"), (field_out, "field_out")):
            if t is not None and (not t.is_cuda or t.dtype != torch.float64 or
                                  not t.is_contiguous() or t.numel() < nx):
                raise ValueError(f"poisson_shift: {nm} must be a contiguous float64 device "
                                 f"tensor of >= {nx} elements")
        _check(getattr(lib(), entry)(self.handle, _ptr(mass), _ptr(hi), float(hx), float(hv),
                                     float(dt), _ptr(shift_out),
                                     None if field_out is None else _ptr(field_out)), entry)
        return shift_out

    def vlasov_poisson_steps(self, nsteps, shift_x, hx, hv, dt, state0, state1, shift_v=None):
        """nsteps self-consistent Strang steps (sldg_vlasov_poisson_steps);
        returns the index (0 or 1) of the state holding the result."""
        import torch
        self._check_shift(shift_x, 2, "vlasov_poisson_steps")
        self._check_state(*state0, "vlasov_poisson_steps state0")
        self._check_state(*state1, "vlasov_poisson_steps state1")
        if shift_v is None:
            shift_v = torch.empty(self.ncells[0], dtype=torch.float64, device=state0[0].device)
        self._check_shift(shift_v, 1, "vlasov_poisson_steps")
        res = ctypes.c_int(-1)
        _check(lib().sldg_vlasov_poisson_steps(self.handle, int(nsteps), _ptr(shift_x), float(hx),
                                               float(hv), float(dt), _ptr(shift_v),
                                               _ptr(state0[0]), _ptr(state0[1]),
                                               _ptr(state1[0]), _ptr(state1[1]),
                                               ctypes.byref(res)), "sldg_vlasov_poisson_steps")
        return res.value

    # --- self-consistent field of (x1, x2, v1, v2) problems ----------------

    def _check_xtable(self, t, n, what):
        import torch
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or
                              not t.is_contiguous() or t.numel() < n):
            raise ValueError(f"{what} must be a contiguous float64 device tensor of >= {n} "
                             f"elements")

    def poisson_shift_2d(self, mass, hi, h, dt, shift_v1=None, shift_v2=None, field_out=None):
        """The v1- and v2-sweep displacements E_1 dt / h_v1, E_2 dt / h_v2 of
        the state's field (sldg_poisson_shift_2d); h = (h_x1, h_x2, h_v1,
        h_v2).  Returns (shift_v1, shift_v2), device float64 [N1 N2] each."""
        import torch
        self._check_state(mass, hi, "poisson_shift_2d")
        if self.ndim != 4:
            raise ValueError("poisson_shift_2d needs an (x1, x2, v1, v2) plan")
        nxx = self.ncells[0] * self.ncells[1]
        if shift_v1 is None:
            shift_v1 = torch.empty(nxx, dtype=torch.float64, device=mass.device)
        if shift_v2 is None:
            shift_v2 = torch.empty(nxx, dtype=torch.float64, device=mass.device)
        self._check_xtable(shift_v1, nxx, "poisson_shift_2d: shift_v1")
        self._check_xtable(shift_v2, nxx, "poisson_shift_2d: shift_v2")
        self._check_xtable(field_out, 2 * nxx, "poisson_shift_2d: field_out")
        hh = (ctypes.c_double * 4)(*[float(x) for x in h])
        _check(lib().sldg_poisson_shift_2d(self.handle, _ptr(mass), _ptr(hi), hh, float(dt),
                                           _ptr(shift_v1), _ptr(shift_v2),
                                           None if field_out is None else _ptr(field_out)),
               "sldg_poisson_shift_2d")
        return shift_v1, shift_v2

    def vlasov_poisson_steps_2d2v(self, nsteps, shift_x1, shift_x2, h, dt, state0, state1,
                                  shift_v1=None, shift_v2=None):
        """nsteps self-consistent Strang steps of an (x1, x2, v1, v2) plan
        (sldg_vlasov_poisson_steps_2d2v); returns the index (0 or 1) of the
        state holding the result."""
        import torch
        if self.ndim != 4:
            raise ValueError("vlasov_poisson_steps_2d2v needs an (x1, x2, v1, v2) plan")
        self._check_shift(shift_x1, 4, "vlasov_poisson_steps_2d2v")
        self._check_shift(shift_x2, 8, "vlasov_poisson_steps_2d2v")
        self._check_state(*state0, "vlasov_poisson_steps_2d2v state0")
        self._check_state(*state1, "vlasov_poisson_steps_2d2v state1")
        nxx = self.ncells[0] * self.ncells[1]
        if shift_v1 is None:
            shift_v1 = torch.empty(nxx, dtype=torch.float64, device=state0[0].device)
        if shift_v2 is None:
            shift_v2 = torch.empty(nxx, dtype=torch.float64, device=state0[0].device)
        self._check_shift(shift_v1, 3, "vlasov_poisson_steps_2d2v")
        self._check_shift(shift_v2, 3, "vlasov_poisson_steps_2d2v")
        hh = (ctypes.c_double * 4)(*[float(x) for x in h])
        res = ctypes.c_int(-1)
        _check(lib().sldg_vlasov_poisson_steps_2d2v(
            self.handle, int(nsteps), _ptr(shift_x1), _ptr(shift_x2), hh, float(dt),
            _ptr(shift_v1), _ptr(shift_v2), _ptr(state0[0]), _ptr(state0[1]), _ptr(state1[0]),
            _ptr(state1[1]), ctypes.byref(res)), "sldg_vlasov_poisson_steps_2d2v")
        return res.value

    # --- launch shapes and the autotuner -----------------------------------

    def set_shape(self, dim, rows, tuples, colwaves=1):
        """Launch shape of the sweeps along `dim` (sldg_plan_set_shape).
        colwaves is 1, 2 or 4, plus the flags SLDG_SHAPE_STAGED (sources
        staged through LDS) and SLDG_SHAPE_MEMORDER (tiles in memory order)."""
        _check(lib().sldg_plan_set_shape(self.handle, int(dim), int(rows), int(tuples),
                                         int(colwaves)), "sldg_plan_set_shape")

    def shape(self, dim):
        r, t, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().sldg_plan_get_shape(self.handle, int(dim), ctypes.byref(r), ctypes.byref(t),
                                         ctypes.byref(c)), "sldg_plan_get_shape")
        return {"rows": r.value, "tuples": t.value, "colwaves": c.value}

    def shapes(self):
        return [self.shape(d) for d in range(self.ndim)]

    def sweep_form(self, dim, dep_mask, state_in, state_out):
        """Kernel form of a sweep along `dim` with the current shape and these
        buffers (sldg_plan_sweep_form): one of SWEEP_FORMS."""
        f = ctypes.c_int()
        _check(lib().sldg_plan_sweep_form(self.handle, int(dim), int(dep_mask),
                                          _ptr(state_in[0]), _ptr(state_in[1]),
                                          _ptr(state_out[0]), _ptr(state_out[1]),
                                          ctypes.byref(f)), "sldg_plan_sweep_form")
        return SWEEP_FORMS[f.value]

    def tune(self, seq, state0, state1, reps=3):
        """Time the candidate shapes of every swept dimension from state0 into
        state1 (overwritten) and keep the fastest (sldg_plan_tune).  Returns
        the per-dimension shapes and the kept time of each sweep of seq."""
        descs = (SweepDesc * max(1, len(seq)))()
        for q, (dim, mask, shift) in enumerate(seq):
            self._check_shift(shift, mask, "tune")
            descs[q] = SweepDesc(int(dim), int(mask), _ptr(shift))
        self._check_state(*state0[:2], "tune state0")
        self._check_state(*state1[:2], "tune state1")
        ms = (ctypes.c_double * max(1, len(seq)))()
        _check(lib().sldg_plan_tune(self.handle, descs, len(seq), _ptr(state0[0]),
                                    _ptr(state0[1]), _ptr(state1[0]), _ptr(state1[1]), int(reps),
                                    ms), "sldg_plan_tune")
        return self.shapes(), [ms[q] for q in range(len(seq))]

    def signature(self, seq):
        """Shape signature (grid, degree, tier, FP64 modes, swept dims and
        masks) for tuning caches."""
        import hashlib
        import json
        txt = json.dumps([list(self.ncells), self.k, self.tier, self.ndouble,
                          [(int(d), int(m)) for d, m, _ in seq]])
        return hashlib.sha256(txt.encode()).hexdigest()[:24]

    def tune_cached(self, path, seq, state0, state1, reps=3):
        """Shapes from the JSON cache at `path` if it holds this plan's
        signature, else tune now and store them.  Returns (shapes, cached)."""
        import json
        cache = {}
        if os.path.exists(path):
            with open(path) as f:
                cache = json.load(f)
        key = self.signature(seq)
        if key in cache:
            for d, sh in enumerate(cache[key]):
                self.set_shape(d, sh["rows"], sh["tuples"], sh["colwaves"])
            return cache[key], True
        shapes, _ = self.tune(seq, state0, state1, reps)
        cache[key] = shapes
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
        return shapes, False

    # --- FP16 storage with per-plane power-of-two scaling ------------------

    def empty_scale(self, device="cuda"):
        """An uninitialised scale block: int32 [2, n_hi], row 0 the storage
        exponents, row 1 the absmax values (float32 bits; see scale_parts)."""
        import torch
        return torch.empty((2, self.n_hi), dtype=torch.int32, device=device)

    @staticmethod
    def scale_parts(scale):
        """(exponents int32 [n_hi], absmax float32 [n_hi]) views of a scale block."""
        return scale[0], scale[1].view(__import__("torch").float32)

    def _check_hi(self, hi, what):
        import torch
        if not isinstance(hi, torch.Tensor) or not hi.is_cuda or \
                hi.dtype != hi_dtype(self.tier) or not hi.is_contiguous() or \
                hi.numel() * hi.element_size() < self.hi_bytes():
            raise ValueError(f"{what}: hi must be a contiguous {hi_dtype(self.tier)} device "
                             f"tensor of {self.hi_bytes()} bytes")

    def _check_scale(self, scale, what):
        import torch
        if not isinstance(scale, torch.Tensor) or not scale.is_cuda or \
                scale.dtype != torch.int32 or not scale.is_contiguous() or \
                scale.numel() < 2 * self.n_hi:
            raise ValueError(f"{what}: scale block must be a contiguous int32 device tensor of "
                             f">= {2 * self.n_hi} elements")

    def set_scale_headroom(self, binades):
        _check(lib().sldg_set_scale_headroom(self.handle, int(binades)), "sldg_set_scale_headroom")

    def scaled_import(self, hi64, hi, scale):
        """Scaled FP16 planes and scale block from FP64 values [n_hi, cells]."""
        import torch
        if not isinstance(hi64, torch.Tensor) or not hi64.is_cuda or \
                hi64.dtype != torch.float64 or not hi64.is_contiguous() or \
                hi64.numel() < self.n_hi * self.cells:
            raise ValueError("scaled_import: hi64 must be contiguous float64 [n_hi, cells] on the device")
        self._check_hi(hi, "scaled_import")
        self._check_scale(scale, "scaled_import")
        _check(lib().sldg_scaled_import(self.handle, _ptr(hi64), _ptr(hi), _ptr(scale)),
               "sldg_scaled_import")

    def scaled_export(self, hi, scale, hi64=None):
        """The FP64 values a scaled FP16 state's narrow planes represent."""
        import torch
        self._check_hi(hi, "scaled_export")
        self._check_scale(scale, "scaled_export")
        if hi64 is None:
            hi64 = torch.empty((self.n_hi, self.cells), dtype=torch.float64, device=hi.device)
        _check(lib().sldg_scaled_export(self.handle, _ptr(hi), _ptr(scale), _ptr(hi64)),
               "sldg_scaled_export")
        return hi64

    def advect_dim_scaled(self, dim, shift, dep_mask, in_mass, in_hi, in_scale, out_mass,
                          out_hi, out_scale):
        """One projection sweep of scaled FP16 states (sldg_advect_dim_scaled)."""
        self._check_shift(shift, dep_mask, "advect_dim_scaled")
        self._check_state(in_mass, in_hi, "advect_dim_scaled input")
        self._check_state(out_mass, out_hi, "advect_dim_scaled output")
        self._check_scale(in_scale, "advect_dim_scaled input")
        self._check_scale(out_scale, "advect_dim_scaled output")
        _check(lib().sldg_advect_dim_scaled(self.handle, int(dim), _ptr(shift), int(dep_mask),
                                            _ptr(in_mass), _ptr(in_hi), _ptr(in_scale),
                                            _ptr(out_mass), _ptr(out_hi), _ptr(out_scale)),
               "sldg_advect_dim_scaled")

    def split_steps_scaled(self, seq, nsteps, state0, state1):
        """split_steps on scaled FP16 states (mass, hi, scale); returns the
        index of the state that holds the result."""
        descs = (SweepDesc * max(1, len(seq)))()
        for q, (dim, mask, shift) in enumerate(seq):
            self._check_shift(shift, mask, "split_steps_scaled")
            descs[q] = SweepDesc(int(dim), int(mask), _ptr(shift))
        for i, st in enumerate((state0, state1)):
            self._check_state(st[0], st[1], f"split_steps_scaled state{i}")
            self._check_scale(st[2], f"split_steps_scaled state{i}")
        res = ctypes.c_int(-1)
        _check(lib().sldg_split_steps_scaled(self.handle, descs, len(seq), int(nsteps),
                                             _ptr(state0[0]), _ptr(state0[1]), _ptr(state0[2]),
                                             _ptr(state1[0]), _ptr(state1[1]), _ptr(state1[2]),
                                             ctypes.byref(res)), "sldg_split_steps_scaled")
        return res.value

    def mass(self, mass):
        """Sum of the mass array as a double-double (hi, lo) (sldg_mass);
        synchronises the plan's stream."""
        import torch
        if mass.dtype != torch.float64 or not mass.is_cuda or not mass.is_contiguous() or \
                mass.numel() < self.cells:
            raise ValueError("mass must be a contiguous float64 device tensor")
        out = (ctypes.c_double * 2)()
        _check(lib().sldg_mass(self.handle, _ptr(mass), out), "sldg_mass")
        return out[0], out[1]

    def mass_device(self, mass, out):
        """Double-double mass sum into the device tensor out[2] (sldg_mass_device);
        asynchronous."""
        import torch
        if mass.dtype != torch.float64 or not mass.is_cuda or not mass.is_contiguous() or \
                mass.numel() < self.cells:
            raise ValueError("mass must be a contiguous float64 device tensor")
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 2:
            raise ValueError("out must be a float64 device tensor of >= 2 elements")
        _check(lib().sldg_mass_device(self.handle, _ptr(mass), _ptr(out)), "sldg_mass_device")

    def timing_enable(self, enable=True):
        """Bracket every later sweep kernel with HIP events (sldg_timing_enable)."""
        _check(lib().sldg_timing_enable(self.handle, 1 if enable else 0), "sldg_timing_enable")

    def timing_read(self, dim):
        """(launches, total ms) of the timed sweep kernels along `dim`
        (-1: dimension 0, -2: dimensions > 0) (sldg_timing_read)."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().sldg_timing_read(self.handle, int(dim), ctypes.byref(n), ctypes.byref(ms)),
               "sldg_timing_read")
        return n.value, ms.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().sldg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_candidates(strided):
    """The launch shapes sldg_plan_tune tries for dimension-0 (False) or
    strided (True) sweeps, as dicts."""
    out = []
    i = 0
    while True:
        r, t, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        st = lib().sldg_tune_candidate(1 if strided else 0, i, ctypes.byref(r), ctypes.byref(t),
                                       ctypes.byref(c))
        if st != SLDG_OK:
            return out
        out.append({"rows": r.value, "tuples": t.value, "colwaves": c.value})
        i += 1


def device_plane_copy(src, dst, plane_bytes, nplanes, planes_per_thread, stream=None):
    """Plane copy of nplanes planes (sldg_device_plane_copy): the reference
    bandwidth of the sweeps' access pattern."""
    if src.numel() * src.element_size() < plane_bytes * nplanes or \
            dst.numel() * dst.element_size() < plane_bytes * nplanes:
        raise ValueError("device_plane_copy: buffers smaller than plane_bytes * nplanes")
    st = _current_stream() if stream is None else stream
    _check(lib().sldg_device_plane_copy(_ptr(src), _ptr(dst), int(plane_bytes), int(nplanes),
                                        int(planes_per_thread), ctypes.c_void_p(st)),
           "sldg_device_plane_copy")


def set_device_alloc_limit(nbytes):
    """Cap on the device bytes the library holds for its own buffers
    (sldg_set_device_alloc_limit); None or -1 removes it."""
    _check(lib().sldg_set_device_alloc_limit(-1 if nbytes is None else int(nbytes)),
           "sldg_set_device_alloc_limit")


def device_alloc_bytes():
    """Device bytes the library holds for its own buffers now."""
    return int(lib().sldg_device_alloc_bytes())


def device_copy(src, dst, nbytes=None, stream=None):
    """Plain device copy of nbytes (sldg_device_copy): the reference bandwidth."""
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if nbytes > src.numel() * src.element_size() or nbytes > dst.numel() * dst.element_size():
        raise ValueError("copy larger than the buffers")
    if not (src.is_cuda and dst.is_cuda):
        raise ValueError("device_copy needs device tensors")
    stream = _current_stream() if stream is None else stream
    _check(lib().sldg_device_copy(_ptr(src), _ptr(dst), nbytes, ctypes.c_void_p(stream)),
           "sldg_device_copy")


# Function names of the C ABI, for callers that prefer them.
def plan(ncells, k, tier="fp32", stream=None):
    return Plan(ncells, k, tier, stream)


def plan_destroy(p):
    p.close()


def advect_dim(p, dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi):
    p.advect_dim(dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi)


def advect_dim_adjoint(p, dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi):
    p.advect_dim_adjoint(dim, shift, dep_mask, in_mass, in_hi, out_mass, out_hi)


def split_steps(p, seq, nsteps, state0, state1):
    return p.split_steps(seq, nsteps, state0, state1)


def mass(p, mass_plane):
    return p.mass(mass_plane)


def line_tables(p, sigma, period):
    return p.line_tables(sigma, period)
