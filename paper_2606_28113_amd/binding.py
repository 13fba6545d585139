"""ctypes binding of libsgspm.so: the C ABI of include/sgspm.h, same names, no logic."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libsgspm.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENUMERIC = 0, -1, -2, -3, -4, -5
TERM_EXCHANGE, TERM_ANISO, TERM_STRAY, TERM_ZEEMAN = 1, 2, 4, 8
TERM_ALL = 15
UNITS_SI, UNITS_REDUCED = 0, 1
FP32, FP64 = 0, 1
SCHEME_SGS, SCHEME_GS, SCHEME_SGS_FF = 0, 1, 2

EXPORTS = ("sgspm_validate", "sgspm_reduced_constants", "sgspm_plan", "sgspm_step", "sgspm_steps",
           "sgspm_step_batch", "sgspm_steps_batch", "sgspm_energy_batch",
           "sgspm_step_spectral_radius",
           "sgspm_energy", "sgspm_unit_error",
           "sgspm_field", "sgspm_stray", "sgspm_heat_solve", "sgspm_adjoint_step",
           "sgspm_adjoint_step_noalloc", "sgspm_tape_bytes", "sgspm_step_taped", "sgspm_adjoint_step_taped",
           "sgspm_demag_tensor", "sgspm_timing",
           "sgspm_timing_read", "sgspm_check", "sgspm_destroy", "sgspm_last_error")
KERNEL_CLASSES = ("row_fwd", "row_fwd512", "row_inv", "row_inv512", "col_dct", "yz_solve", "yz_reg",
                  "col_fft", "fft512", "conv", "conv64", "other")


class SGSPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgspm error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("units", ctypes.c_int32),
                ("A", ctypes.c_double), ("Ms", ctypes.c_double), ("Ku", ctypes.c_double),
                ("eps", ctypes.c_double), ("Q", ctypes.c_double),
                ("dt", ctypes.c_double),
                ("terms", ctypes.c_uint32),
                ("precision", ctypes.c_int32),
                ("scheme", ctypes.c_int32),
                ("batch", ctypes.c_int32)]


def _load():
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is missing: build it with __graft_entry__.build() "
                          "or python paper_2606_28113_amd/build.py (no CPU fallback exists)")
    L = ctypes.CDLL(lib_path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.sgspm_validate.argtypes = [ctypes.POINTER(Params)]
    L.sgspm_reduced_constants.argtypes = [ctypes.POINTER(Params), dp]
    L.sgspm_plan.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.sgspm_step.argtypes = [vp, vp, ctypes.c_double, dp, vp]
    L.sgspm_step_spectral_radius.argtypes = [vp, vp, ctypes.c_double, dp, vp, dp]
    L.sgspm_steps.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, dp]
    L.sgspm_step_batch.argtypes = [vp, vp, dp, dp]
    L.sgspm_steps_batch.argtypes = [vp, vp, ctypes.c_int, dp, dp]
    L.sgspm_energy_batch.argtypes = [vp, vp, dp, dp]
    L.sgspm_energy.argtypes = [vp, vp, dp, dp]
    L.sgspm_unit_error.argtypes = [vp, vp, dp]
    L.sgspm_field.argtypes = [vp, vp, dp, vp]
    L.sgspm_stray.argtypes = [vp, vp, vp]
    L.sgspm_heat_solve.argtypes = [vp, vp, ctypes.c_double, vp]
    L.sgspm_adjoint_step.argtypes = [vp, vp, ctypes.c_double, dp, vp, vp]
    L.sgspm_adjoint_step_noalloc.argtypes = [vp, vp, ctypes.c_double, dp, vp, vp]
    L.sgspm_tape_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.sgspm_step_taped.argtypes = [vp, vp, ctypes.c_double, dp, vp]
    L.sgspm_adjoint_step_taped.argtypes = [vp, vp, ctypes.c_double, dp, vp, vp, vp]
    L.sgspm_demag_tensor.argtypes = [vp, ctypes.c_int, vp]
    L.sgspm_timing.argtypes = [vp, ctypes.c_int]
    L.sgspm_timing_read.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
    L.sgspm_check.argtypes = [vp]
    L.sgspm_destroy.argtypes = [vp]
    L.sgspm_last_error.argtypes = []
    L.sgspm_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-1]:
        getattr(L, name).restype = ip
    return L


lib = _load()


def _check(rc):
    if rc != OK:
        raise SGSPMError(rc, lib.sgspm_last_error().decode())


def make_params(nx, ny, nz, dx, dy, dz, dt, units=UNITS_SI, A=0.0, Ms=1.0, Ku=0.0, eps=0.0, Q=0.0,
                terms=TERM_ALL, precision=FP32, scheme=SCHEME_SGS, batch=0):
    return Params(nx, ny, nz, dx, dy, dz, units, A, Ms, Ku, eps, Q, dt, terms, precision, scheme, batch)


def validate(**kw):
    p = make_params(**kw)
    _check(lib.sgspm_validate(ctypes.byref(p)))


def reduced_constants(**kw):
    """(eps, Q, dt_reduced, field scale per tesla, energy scale) of a parameter set."""
    p = make_params(**kw)
    out = (ctypes.c_double * 5)()
    _check(lib.sgspm_reduced_constants(ctypes.byref(p), out))
    return tuple(out)


def _d3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


class Plan:
    """A plan on the current torch CUDA stream (fixed at creation).

    Keyword arguments are the fields of sgspm_params (see make_params).
    Field tensors: CUDA, contiguous, shape (3, nz, ny, nx), dtype float32 for
    FP32 plans and float64 for FP64 plans; a batched plan (batch = B >= 2) takes
    (3, B, nz, ny, nx) and the *_batch methods.
    """

    def __init__(self, **kw):
        import torch
        self.kw = dict(kw)
        self.params = make_params(**kw)
        self.n = (self.params.nx, self.params.ny, self.params.nz)
        self.dtype = torch.float64 if self.params.precision == FP64 else torch.float32
        self.stream = torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        _check(lib.sgspm_plan(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(self._h)))

    @property
    def batch(self):
        return max(1, self.params.batch)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (3, self.batch, nz, ny, nx) if self.batch > 1 else (3, nz, ny, nx)

    def _runs(self, alpha, h_e):
        B = self.batch
        a = [float(x) for x in alpha]
        h = [float(x) for row in h_e for x in row]
        if len(a) != B or len(h) != 3 * B:
            raise ValueError(f"alpha needs {B} values and h_e {B} rows of 3")
        return (ctypes.c_double * B)(*a), (ctypes.c_double * (3 * B))(*h)

    def step_batch(self, m, alpha, h_e):
        """One step of every run of a batched plan: run b with alpha[b] and h_e[b]."""
        a, h = self._runs(alpha, h_e)
        _check(lib.sgspm_step_batch(self._h, self._ptr(m, self.shape, "m"), a, h))

    def steps_batch(self, m, nsteps, alpha, h_e):
        """nsteps batched steps with constant per-run alpha and h_e (captured HIP graph)."""
        a, h = self._runs(alpha, h_e)
        _check(lib.sgspm_steps_batch(self._h, self._ptr(m, self.shape, "m"), int(nsteps), a, h))

    def energy_batch(self, m, h_e):
        """Energies of every run: a list of dicts as energy() returns."""
        B = self.batch
        _, h = self._runs([0.0] * B, h_e)
        out = (ctypes.c_double * (5 * B))()
        _check(lib.sgspm_energy_batch(self._h, self._ptr(m, self.shape, "m"), h, out))
        keys = ("total", "exchange", "anisotropy", "stray", "zeeman")
        return [dict(zip(keys, list(out[5 * b:5 * b + 5]))) for b in range(B)]

    def _ptr(self, t, shape=None, name="tensor"):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != self.dtype:
            raise ValueError(f"{name} must be a contiguous CUDA {self.dtype} tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def step(self, m, alpha, h_e, src=None):
        s = None if src is None else self._ptr(src, self.shape, "src")
        _check(lib.sgspm_step(self._h, self._ptr(m, self.shape, "m"), float(alpha), _d3(h_e), s))

    def steps(self, m, nsteps, alpha, h_e):
        """nsteps steps with constant alpha and h_e, replayed from a captured HIP graph."""
        _check(lib.sgspm_steps(self._h, self._ptr(m, self.shape, "m"), int(nsteps), float(alpha), _d3(h_e)))

    def step_spectral_radius(self, m, alpha, h_e, src=None):
        """One step (as step) and (rho(G_GS), rho(G_SGS)) of its sweep matrices."""
        s = None if src is None else self._ptr(src, self.shape, "src")
        out = (ctypes.c_double * 2)()
        _check(lib.sgspm_step_spectral_radius(self._h, self._ptr(m, self.shape, "m"), float(alpha), _d3(h_e), s, out))
        return out[0], out[1]

    def energy(self, m, h_e):
        out = (ctypes.c_double * 5)()
        _check(lib.sgspm_energy(self._h, self._ptr(m, self.shape, "m"), _d3(h_e), out))
        return dict(zip(("total", "exchange", "anisotropy", "stray", "zeeman"), list(out)))

    def unit_error(self, m):
        """max over cells of | |m| - 1 |."""
        out = ctypes.c_double()
        _check(lib.sgspm_unit_error(self._h, self._ptr(m, self.shape, "m"), ctypes.byref(out)))
        return out.value

    def field(self, m, h_e, out=None):
        import torch
        out = torch.empty_like(m) if out is None else out
        _check(lib.sgspm_field(self._h, self._ptr(m, self.shape, "m"), _d3(h_e), self._ptr(out, self.shape, "out")))
        return out

    def stray(self, m, out=None):
        import torch
        out = torch.empty_like(m) if out is None else out
        _check(lib.sgspm_stray(self._h, self._ptr(m, self.shape, "m"), self._ptr(out, self.shape, "out")))
        return out

    def heat_solve(self, r, s, out=None):
        import torch
        out = torch.empty_like(r) if out is None else out
        shp = self.shape[1:]
        _check(lib.sgspm_heat_solve(self._h, self._ptr(r, shp, "r"), float(s), self._ptr(out, shp, "out")))
        return out

    def adjoint_step(self, m_n, alpha, h_e, lam, grad):
        import torch
        if not grad.is_cuda or grad.dtype != torch.float64 or grad.numel() != 4 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous CUDA float64 tensor of 4 values")
        _check(lib.sgspm_adjoint_step(self._h, self._ptr(m_n, self.shape, "m_n"), float(alpha), _d3(h_e),
                                      self._ptr(lam, self.shape, "lam"), ctypes.c_void_p(grad.data_ptr())))

    def adjoint_step_noalloc(self, m_n, alpha, h_e, lam, grad):
        import torch
        if not grad.is_cuda or grad.dtype != torch.float64 or grad.numel() != 4 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous CUDA float64 tensor of 4 values")
        _check(lib.sgspm_adjoint_step_noalloc(self._h, self._ptr(m_n, self.shape, "m_n"), float(alpha), _d3(h_e),
                                              self._ptr(lam, self.shape, "lam"), ctypes.c_void_p(grad.data_ptr())))

    def tape_bytes(self):
        """Device bytes of one step's tape (step_taped / adjoint_step_taped)."""
        n = ctypes.c_size_t()
        _check(lib.sgspm_tape_bytes(self._h, ctypes.byref(n)))
        return n.value

    def new_tapes(self, count):
        """Device storage for `count` step tapes: a uint8 tensor, one row per tape."""
        import torch
        return torch.empty((int(count), self.tape_bytes()), dtype=torch.uint8, device="cuda")

    def _tape_ptr(self, tape):
        import torch
        if (not tape.is_cuda or not tape.is_contiguous() or tape.dtype != torch.uint8
                or tape.numel() < self.tape_bytes()):
            raise ValueError(f"tape must be a contiguous CUDA uint8 tensor of at least {self.tape_bytes()} bytes")
        return ctypes.c_void_p(tape.data_ptr())

    def step_taped(self, m, alpha, h_e, tape):
        """One step in place (as step) that also writes its tape."""
        _check(lib.sgspm_step_taped(self._h, self._ptr(m, self.shape, "m"), float(alpha), _d3(h_e),
                                    self._tape_ptr(tape)))

    def adjoint_step_taped(self, m_n, alpha, h_e, tape, lam, grad):
        """adjoint_step from the tape step_taped wrote for the same m_n, alpha and h_e."""
        import torch
        if not grad.is_cuda or grad.dtype != torch.float64 or grad.numel() != 4 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous CUDA float64 tensor of 4 values")
        _check(lib.sgspm_adjoint_step_taped(self._h, self._ptr(m_n, self.shape, "m_n"), float(alpha), _d3(h_e),
                                            self._tape_ptr(tape), self._ptr(lam, self.shape, "lam"),
                                            ctypes.c_void_p(grad.data_ptr())))

    def demag_tensor(self, comp, out=None):
        """Real-space FP64 tensor component comp (0..5 = xx yy zz xy xz yz) on the padded grid (Pz, Py, Px)."""
        import torch
        P = tuple(2 * n if n > 1 else 1 for n in self.n)
        shp = (P[2], P[1], P[0])
        out = torch.empty(shp, dtype=torch.float64, device="cuda") if out is None else out
        if not out.is_cuda or out.dtype != torch.float64 or not out.is_contiguous() or tuple(out.shape) != shp:
            raise ValueError(f"out must be a contiguous CUDA float64 tensor of shape {shp}")
        _check(lib.sgspm_demag_tensor(self._h, int(comp), ctypes.c_void_p(out.data_ptr())))
        return out

    def timing(self, enable=True):
        _check(lib.sgspm_timing(self._h, 1 if enable else 0))

    def timing_read(self):
        """{class: (ms, launch-level bytes, launches)} since the last enable / read."""
        n = len(KERNEL_CLASSES)
        ms, by, cnt = (ctypes.c_double * n)(), (ctypes.c_double * n)(), (ctypes.c_int64 * n)()
        _check(lib.sgspm_timing_read(self._h, ms, by, cnt))
        return {k: (ms[i], by[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def check(self):
        _check(lib.sgspm_check(self._h))

    def close(self):
        if self._h:
            lib.sgspm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
