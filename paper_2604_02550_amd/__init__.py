"""Python binding of libacse.so, the MI355X ACSE residual library.

Argument marshalling only: every step of the residual, update and energy runs
in the HIP kernels behind the C ABI of ``include/acse.h``.  PyTorch provides
device memory and the stream.  If the shared library is missing the import
fails; there is no CPU fallback.

    import paper_2604_02550_amd as acse
    ctx = acse.Context(r_max=50)
    R_aa, R_ab, norm2 = ctx.residual(h, V, d1, d2aa, d2ab, n_alpha, precision="fp64")
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacse.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2604_02550_amd/build.py "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

FP64, FP32, BF16X3, INT8CRT = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "int8crt": INT8CRT}
STATUS = {0: "ACSE_OK", 1: "ACSE_ERR_ARG", 2: "ACSE_ERR_SHAPE", 3: "ACSE_ERR_ALIGN",
          4: "ACSE_ERR_UNSUPPORTED", 5: "ACSE_ERR_NOMEM", 6: "ACSE_ERR_HIP",
          7: "ACSE_ERR_NONFINITE"}

# Every function declared in include/acse.h.
EXPORTS = ("acse_create", "acse_destroy", "acse_set_stream", "acse_residual", "acse_update_map",
           "acse_energy", "acse_step", "acse_status_str", "acse_last_error",
           "acse_workspace_bytes", "acse_profile_enable", "acse_profile_read", "acse_autotune",
           "acse_residual_vjp", "acse_energy_vjp", "acse_residual_batched",
           "acse_autotune_batched", "acse_solve", "acse_residual_noalloc", "acse_residual_spin",
           "acse_step_spin", "acse_energy_spin", "acse_solve_spin")
NUM_TILE_CONFIGS = 3
NUM_STAGES = 8
STAGES = ("rdm_operands", "fold", "transforms", "gemm", "assembly", "step_tail", "ny_share", "ny_gemm")


class Problem(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("n_alpha", ctypes.c_int32), ("n_beta", ctypes.c_int32),
                ("h", ctypes.c_void_p), ("V", ctypes.c_void_p), ("d1", ctypes.c_void_p),
                ("d2aa", ctypes.c_void_p), ("d2ab", ctypes.c_void_p)]


class ProblemSpin(ctypes.Structure):
    """acse_problem_spin: a state of any S_z (alpha and beta 1-RDMs, the three 2-RDM blocks)."""
    _fields_ = [("r", ctypes.c_int32), ("n_alpha", ctypes.c_int32), ("n_beta", ctypes.c_int32),
                ("h", ctypes.c_void_p), ("V", ctypes.c_void_p), ("d1a", ctypes.c_void_p), ("d1b", ctypes.c_void_p),
                ("d2aa", ctypes.c_void_p), ("d2bb", ctypes.c_void_p), ("d2ab", ctypes.c_void_p)]


class ProfileData(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NUM_STAGES), ("count", ctypes.c_int64 * NUM_STAGES)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("active", ctypes.c_void_p), ("tile", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reconstruction", ctypes.c_int32), ("ny_sigma", ctypes.c_void_p),
                ("moduli", ctypes.c_int32)]


RECON_V, RECON_NY = 0, 1


FLAG_GENERAL_KERNELS = 1
FLAG_CHECK_INPUTS = 2
FLAG_BATCH_PERSISTENT = 4

EULER_FIXED, EULER_BACKTRACK, EULER_QUADRATIC = 0, 1, 2
CONTROLS = {"fixed": EULER_FIXED, "backtrack": EULER_BACKTRACK, "quadratic": EULER_QUADRATIC}
STOP_REASONS = ("max_iter", "converged", "energy_rose", "norm_rose")


class SolveOptions(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("de_tol", ctypes.c_double), ("eps_max", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("control", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Trial(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("energy", ctypes.c_double), ("norm2", ctypes.c_double),
                ("step", ctypes.c_int32), ("accepted", ctypes.c_int32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("energy0", ctypes.c_double), ("norm2_0", ctypes.c_double),
                ("energy", ctypes.c_double), ("norm2", ctypes.c_double), ("eps", ctypes.c_double),
                ("iterations", ctypes.c_int32), ("trials", ctypes.c_int32), ("maps", ctypes.c_int32),
                ("stop", ctypes.c_int32)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_sig = {
    "acse_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.c_int32]),
    "acse_destroy": (ctypes.c_int, [_P]),
    "acse_set_stream": (ctypes.c_int, [_P, _P]),
    "acse_residual": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options), _P, _P, _D]),
    "acse_update_map": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options), _P, _P,
                                       _P, _P]),
    "acse_energy": (ctypes.c_int, [_P, ctypes.POINTER(Problem), _D]),
    "acse_step": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.c_double,
                                 ctypes.POINTER(Options), _P, _P, _P, _P, _D, _D]),
    "acse_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "acse_last_error": (ctypes.c_char_p, [_P]),
    "acse_workspace_bytes": (ctypes.c_int64, [_P]),
    "acse_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "acse_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(ProfileData)]),
    "acse_autotune": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                     ctypes.POINTER(ctypes.c_int32), _D]),
    "acse_residual_vjp": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                         _P, _P, _P, _P, _P, _P, _P]),
    "acse_energy_vjp": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.c_double,
                                       _P, _P, _P, _P]),
    "acse_residual_batched": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Problem),
                                             ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.POINTER(ctypes.c_void_p), _D]),
    "acse_autotune_batched": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(Problem),
                                             ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int32),
                                             _D]),
    "acse_residual_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options), _P, _P,
                                             _P]),
    "acse_residual_spin": (ctypes.c_int, [_P, ctypes.POINTER(ProblemSpin), ctypes.POINTER(Options), _P, _P, _P,
                                          _D]),
    "acse_step_spin": (ctypes.c_int, [_P, ctypes.POINTER(ProblemSpin), ctypes.c_double, ctypes.POINTER(Options),
                                      _P, _P, _P, _P, _P, _P, _D, _D]),
    "acse_energy_spin": (ctypes.c_int, [_P, ctypes.POINTER(ProblemSpin), _D]),
    "acse_solve_spin": (ctypes.c_int, [_P, ctypes.POINTER(ProblemSpin), ctypes.POINTER(Options),
                                       ctypes.POINTER(SolveOptions), ctypes.POINTER(SolveResult),
                                       ctypes.POINTER(Trial), ctypes.c_int32]),
    "acse_solve": (ctypes.c_int, [_P, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                  ctypes.POINTER(SolveOptions), ctypes.POINTER(SolveResult),
                                  ctypes.POINTER(Trial), ctypes.c_int32]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class AcseError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, device):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=torch.float64).contiguous()


def _shape(x):
    if isinstance(x, torch.Tensor):
        return tuple(x.shape)
    import numpy as np
    return np.shape(x)


def _numel(x):
    n = 1
    for d in _shape(x):
        n *= int(d)
    return n


def check_problem_shapes(h, V, d1, d2aa, d2ab):
    """r from h; ValueError unless h and d1 are r x r and V, d2aa, d2ab hold r^4
    elements each (the library reads exactly that many through each pointer)."""
    sh = _shape(h)
    if len(sh) != 2 or sh[0] != sh[1] or sh[0] < 1:
        raise ValueError(f"h must be a square r x r array, got shape {sh}")
    r = int(sh[0])
    if _shape(d1) != (r, r):
        raise ValueError(f"d1 must have shape ({r}, {r}), got {_shape(d1)}")
    for name, x in (("V", V), ("d2aa", d2aa), ("d2ab", d2ab)):
        if _numel(x) != r ** 4:
            raise ValueError(f"{name} must hold r^4 = {r ** 4} elements (r = {r}), got shape {_shape(x)}")
    return r


def _check_dev4(t, r, name, device):
    """A caller array the library reads or writes as r^4 FP64 values on the device."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on {device}")
    if t.dtype != torch.float64 or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on {device}")
    if t.numel() != r ** 4:
        raise ValueError(f"{name} must hold r^4 = {r ** 4} elements (r = {r}), got shape {tuple(t.shape)}")


def _check_dev2(t, r, name, device):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != device \
            or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on {device}")
    if t.numel() != r * r:
        raise ValueError(f"{name} must hold r^2 = {r * r} elements (r = {r}), got shape {tuple(t.shape)}")


def _check_opts(opts, r, spin=False):
    """The host arrays of the options must cover the problem: the active mask r
    orbitals, the NY occupations r orbitals (2r spin orbitals, alpha first, for
    the calls on states of any S_z)."""
    for name, n in getattr(opts, "_lens", {}).items():
        want = 2 * r if spin and name == "ny_sigma" else r
        if n is not None and n != want:
            what = f"2r = {want} spin orbitals" if want != r else f"r = {r} orbitals"
            raise ValueError(f"options.{name} has {n} entries, the problem has {what}")


class Context:
    """One library context: a device, a stream and workspace for r <= r_max."""

    def __init__(self, r_max, device=0, stream=None):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = dev.index or 0
        self.device = torch.device("cuda", idx)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = _lib.acse_create(ctypes.byref(h), idx, ctypes.c_void_p(self.stream.cuda_stream),
                              int(r_max))
        if st != 0:
            raise AcseError(st, "acse_create failed")
        self._h = h
        self.r_max = r_max

    def close(self):
        if getattr(self, "_h", None):
            _lib.acse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self):
        return int(_lib.acse_workspace_bytes(self._h))

    def profile(self, enable=True):
        """Start (clearing totals) or stop HIP-event timing of the library stages."""
        self._check(_lib.acse_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total ms, intervals)} since the last profile(True); synchronises."""
        d = ProfileData()
        self._check(_lib.acse_profile_read(self._h, ctypes.byref(d)))
        return {STAGES[i]: (d.ms[i], d.count[i]) for i in range(NUM_STAGES)}

    def autotune_raw(self, prob, opts):
        """Times every GEMM tile configuration on this problem and caches the best
        for (r, precision); returns (best index, [ms per configuration])."""
        _check_opts(opts, prob.r)
        best = ctypes.c_int32(-1)
        times = (ctypes.c_double * NUM_TILE_CONFIGS)()
        self._check(_lib.acse_autotune(self._h, ctypes.byref(prob), ctypes.byref(opts),
                                       ctypes.byref(best), times))
        return best.value, list(times)

    def _check(self, st):
        if st != 0:
            raise AcseError(st, _lib.acse_last_error(self._h).decode())

    def problem(self, h, V, d1, d2aa, d2ab, n_alpha, n_beta=None):
        """Device copies (float64, contiguous) and the ctypes problem struct."""
        r = check_problem_shapes(h, V, d1, d2aa, d2ab)
        t = [_dev(x, self.device) for x in (h, V, d1, d2aa, d2ab)]
        prob = Problem(r, int(n_alpha), int(n_alpha if n_beta is None else n_beta),
                       *[x.data_ptr() for x in t])
        return prob, t

    @staticmethod
    def options(precision="fp64", active=None, tile=-1, flags=0, sigma=None, moduli=0):
        """acse_options.  ``sigma`` selects the Nakatsuji-Yasuda reconstruction:
        True for the default reference occupations (orbitals below n_alpha
        occupied; for the _spin calls alpha orbitals below n_alpha and beta
        orbitals below n_beta) or a sequence of +1 / -1 per orbital (per spin
        orbital, alpha first, for the _spin calls); None is Valdemoro.
        ``moduli``: modulus count of the "int8crt" precision (0 = 13)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        keep = None
        act = None
        if active is not None:
            keep = (ctypes.c_uint8 * len(active))(*[1 if a else 0 for a in active])
            act = ctypes.cast(keep, ctypes.c_void_p)
        recon, sig, keep_sig = RECON_V, None, None
        if sigma is not None and sigma is not False:
            recon = RECON_NY
            if sigma is not True:
                keep_sig = (ctypes.c_int8 * len(sigma))(*[int(x) for x in sigma])
                sig = ctypes.cast(keep_sig, ctypes.c_void_p)
        o = Options(prec, act, int(tile), int(flags), recon, sig, int(moduli))
        o._keep = (keep, keep_sig)
        o._lens = {"active": None if keep is None else len(keep),
                   "ny_sigma": None if keep_sig is None else len(keep_sig)}
        return o

    def residual_raw(self, prob, opts, R_aa, R_ab, want_norm=True):
        _check_opts(opts, prob.r)
        for name, t in (("R_aa", R_aa), ("R_ab", R_ab)):
            _check_dev4(t, prob.r, name, self.device)
        n2 = ctypes.c_double(0.0)
        self._check(_lib.acse_residual(self._h, ctypes.byref(prob), ctypes.byref(opts), _ptr(R_aa),
                                       _ptr(R_ab), ctypes.byref(n2) if want_norm else None))
        return n2.value

    def residual(self, h, V, d1, d2aa, d2ab, n_alpha, precision="fp64", tile=-1, flags=0, sigma=None,
                 moduli=0):
        """R_aa, R_ab (device, float64) and ||R||^2 of Eq. (4)."""
        prob, keep = self.problem(h, V, d1, d2aa, d2ab, n_alpha)
        r = prob.r
        R_aa = torch.empty((r, r, r, r), dtype=torch.float64, device=self.device)
        R_ab = torch.empty_like(R_aa)
        n2 = self.residual_raw(prob, self.options(precision, None, tile, flags, sigma, moduli), R_aa, R_ab)
        return R_aa, R_ab, n2

    def update_map(self, h, V, d1, d2aa, d2ab, n_alpha, X_aa, X_ab, precision="fp64", tile=-1, flags=0,
                   sigma=None, moduli=0):
        """U = 1/2 <[a+a+aa, sum X a+a+aa]> for anti-Hermitian X (Eq. (9))."""
        prob, keep = self.problem(h, V, d1, d2aa, d2ab, n_alpha)
        for name, x in (("X_aa", X_aa), ("X_ab", X_ab)):
            if _numel(x) != prob.r ** 4:
                raise ValueError(f"{name} must hold r^4 = {prob.r ** 4} elements, got shape {_shape(x)}")
        X_aa, X_ab = _dev(X_aa, self.device), _dev(X_ab, self.device)
        U_aa = torch.empty_like(X_aa)
        U_ab = torch.empty_like(X_ab)
        self._check(_lib.acse_update_map(self._h, ctypes.byref(prob),
                                         ctypes.byref(self.options(precision, None, tile, flags, sigma, moduli)),
                                         _ptr(X_aa), _ptr(X_ab), _ptr(U_aa), _ptr(U_ab)))
        return U_aa, U_ab

    def energy_raw(self, prob):
        e = ctypes.c_double(0.0)
        self._check(_lib.acse_energy(self._h, ctypes.byref(prob), ctypes.byref(e)))
        return e.value

    def energy(self, h, V, d2aa, d2ab, n_alpha):
        """E = Tr(K 2D) (Eq. (2), Eq. (6))."""
        r = h.shape[0]
        prob, keep = self.problem(h, V, torch.zeros(r, r), d2aa, d2ab, n_alpha)
        return self.energy_raw(prob)

    def step_raw(self, prob, eps, opts, R_aa=None, R_ab=None, U_aa=None, U_ab=None, want=True):
        _check_opts(opts, prob.r)
        for name, t in (("R_aa", R_aa), ("R_ab", R_ab), ("U_aa", U_aa), ("U_ab", U_ab)):
            if t is not None:
                _check_dev4(t, prob.r, name, self.device)
        e = ctypes.c_double(0.0)
        n2 = ctypes.c_double(0.0)
        self._check(_lib.acse_step(self._h, ctypes.byref(prob), float(eps), ctypes.byref(opts),
                                   _ptr(R_aa), _ptr(R_ab), _ptr(U_aa), _ptr(U_ab),
                                   ctypes.byref(e) if want else None,
                                   ctypes.byref(n2) if want else None))
        return e.value, n2.value

    def step(self, h, V, d1, d2aa, d2ab, n_alpha, eps=1e-3, precision="fp64", active=None,
             tile=-1, return_ru=False, flags=0, sigma=None, moduli=0):
        """One Euler step of Eq. (9) on device copies; returns a dict with the new
        d1, d2aa, d2ab, the energy after the step and ||R||^2 before it."""
        prob, t = self.problem(h, V, d1, d2aa, d2ab, n_alpha)
        r = prob.r
        extra = {}
        bufs = [None] * 4
        if return_ru:
            bufs = [torch.empty((r, r, r, r), dtype=torch.float64, device=self.device) for _ in range(4)]
        E, n2 = self.step_raw(prob, eps, self.options(precision, active, tile, flags, sigma, moduli), *bufs)
        if return_ru:
            extra = dict(R_aa=bufs[0], R_ab=bufs[1], U_aa=bufs[2], U_ab=bufs[3])
        return dict(d1=t[2], d2aa=t[3], d2ab=t[4], energy=E, norm2=n2, **extra)

    def solve_raw(self, prob, opts, sopts, capacity=256):
        """acse_solve on a prepared problem; returns (SolveResult, [Trial])."""
        _check_opts(opts, prob.r)
        res = SolveResult()
        hist = (Trial * max(1, capacity))()
        self._check(_lib.acse_solve(self._h, ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(sopts),
                                    ctypes.byref(res), hist, int(capacity)))
        return res, [hist[i] for i in range(min(res.trials, capacity))]

    def solve(self, h, V, d1, d2aa, d2ab, n_alpha, eps=1e-3, de_tol=1e-6, max_iter=100,
              control="fixed", max_halvings=8, eps_max=0.0, precision="fp64", active=None, tile=-1,
              flags=0, capacity=256, sigma=None, moduli=0):
        """The Euler iteration of Eq. (9) with the stopping rules of the method
        section on device copies of the inputs (acse_solve).  Returns a dict with
        the final d1, d2aa, d2ab (device), energy/norm2 of the input and returned
        states, iterations, maps, the stop reason, the last accepted step size and
        the trials as (eps, energy, norm2, step, accepted) tuples."""
        prob, t = self.problem(h, V, d1, d2aa, d2ab, n_alpha)
        so = SolveOptions(float(eps), float(de_tol), float(eps_max), int(max_iter),
                          CONTROLS[control] if isinstance(control, str) else int(control),
                          int(max_halvings), 0)
        res, hist = self.solve_raw(prob, self.options(precision, active, tile, flags, sigma, moduli), so,
                                   capacity)
        return dict(d1=t[2], d2aa=t[3], d2ab=t[4], energy0=res.energy0, norm2_0=res.norm2_0,
                    energy=res.energy, norm2=res.norm2, eps=res.eps, iterations=res.iterations,
                    trial_count=res.trials, maps=res.maps, stop=STOP_REASONS[res.stop],
                    trials=[(q.eps, q.energy, q.norm2, q.step, bool(q.accepted)) for q in hist])

    def solve_checkpointed(self, h, V, d1, d2aa, d2ab, n_alpha, path, every=10, max_iter=100, eps=1e-3,
                           **kw):
        """The iteration of ``solve`` in chunks of ``every`` steps.  After each
        chunk the state (1-RDM, 2-RDM blocks, the next step size, the steps
        taken, the lambda trajectory) is written to ``path`` (numpy .npz of
        plain arrays, replaced atomically).  If ``path`` exists the iteration
        resumes from it: the state it holds replaces d1, d2aa and d2ab, and it
        must have been written for the same h, V, electron count and options
        that change the iteration (``checkpoint_tag``; reconstruction, precision,
        active mask, step control and its limits, de_tol), else ValueError.  Each chunk
        starts from the state the previous one returned, so the result is the
        one an uninterrupted ``solve`` reaches.  Returns the dict of the last
        chunk with ``iterations`` counting every chunk's steps, ``trajectory``
        (see ``trajectory``) and ``resumed``."""
        import numpy as np

        tag = checkpoint_tag(h, V, n_alpha, **kw)
        done, resumed = 0, False
        traj = None
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                if str(z["tag"]) != tag:
                    raise ValueError(f"{path} was written for another problem or other iteration options")
                d1, d2aa, d2ab = z["d1"], z["d2aa"], z["d2ab"]
                eps = float(z["eps"])
                done = int(z["iterations"])
                traj = [tuple(row) for row in z["trajectory"]]
                stop = str(z["stop"])
            resumed = True
            if stop != "max_iter" or done >= max_iter:
                return dict(d1=d1, d2aa=d2aa, d2ab=d2ab, iterations=done, trajectory=traj, stop=stop,
                            resumed=True)
        out = None
        while done < max_iter:
            n = min(int(every), max_iter - done)
            out = self.solve(h, V, d1, d2aa, d2ab, n_alpha, eps=eps, max_iter=n, **kw)
            part = trajectory(out)
            if traj is None:
                traj = part
            else:
                lam0 = traj[-1][0]
                traj += [(lam0 + lam, e, lg) for lam, e, lg in part[1:]]
            done += out["iterations"]
            d1, d2aa, d2ab = out["d1"], out["d2aa"], out["d2ab"]
            if out["iterations"]:
                eps = out["eps"]
            tmp = path + ".tmp.npz"
            np.savez(tmp, tag=np.array(tag), d1=_host64(d1), d2aa=_host64(d2aa), d2ab=_host64(d2ab),
                     eps=np.array(eps), iterations=np.array(done), stop=np.array(out["stop"]),
                     trajectory=np.array(traj, dtype=np.float64).reshape(-1, 3))
            os.replace(tmp, path)
            if out["stop"] != "max_iter":
                break
        if out is None:
            return dict(d1=d1, d2aa=d2aa, d2ab=d2ab, iterations=done, trajectory=traj, stop="max_iter",
                        resumed=resumed)
        return dict(out, iterations=done, trajectory=traj, resumed=resumed)

    # ----- states of any S_z (N_alpha != N_beta) --------------------------------
    def problem_spin(self, h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta):
        """Device copies and the ctypes struct of a state of any S_z."""
        r = check_problem_shapes(h, V, d1a, d2aa, d2ab)
        if _shape(d1b) != (r, r):
            raise ValueError(f"d1b must have shape ({r}, {r}), got {_shape(d1b)}")
        if _numel(d2bb) != r ** 4:
            raise ValueError(f"d2bb must hold r^4 = {r ** 4} elements (r = {r}), got shape {_shape(d2bb)}")
        t = [_dev(x, self.device) for x in (h, V, d1a, d1b, d2aa, d2bb, d2ab)]
        prob = ProblemSpin(r, int(n_alpha), int(n_beta), *[x.data_ptr() for x in t])
        return prob, t

    def residual_spin_raw(self, prob, opts, R_aa, R_bb, R_ab, want_norm=True):
        _check_opts(opts, prob.r, spin=True)
        for name, x in (("R_aa", R_aa), ("R_bb", R_bb), ("R_ab", R_ab)):
            _check_dev4(x, prob.r, name, self.device)
        n2 = ctypes.c_double(0.0)
        self._check(_lib.acse_residual_spin(self._h, ctypes.byref(prob), ctypes.byref(opts), _ptr(R_aa), _ptr(R_bb),
                                            _ptr(R_ab), ctypes.byref(n2) if want_norm else None))
        return n2.value

    def residual_spin(self, h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta, tile=-1, flags=0,
                      precision="fp64", moduli=0, sigma=None):
        """R_aa, R_bb, R_ab (device) and ||R||^2 of Eq. (4) for a state of any S_z
        (precision "fp64" or "int8crt"; ``sigma`` as for ``options``)."""
        prob, keep = self.problem_spin(h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta)
        r = prob.r
        R = [torch.empty((r, r, r, r), dtype=torch.float64, device=self.device) for _ in range(3)]
        n2 = self.residual_spin_raw(prob, self.options(precision, None, tile, flags, sigma, moduli), *R)
        return R[0], R[1], R[2], n2

    def step_spin_raw(self, prob, eps, opts, outs=(None,) * 6, want=True):
        _check_opts(opts, prob.r, spin=True)
        for name, x in zip(("R_aa", "R_bb", "R_ab", "U_aa", "U_bb", "U_ab"), outs):
            if x is not None:
                _check_dev4(x, prob.r, name, self.device)
        e = ctypes.c_double(0.0)
        n2 = ctypes.c_double(0.0)
        self._check(_lib.acse_step_spin(self._h, ctypes.byref(prob), float(eps), ctypes.byref(opts),
                                        *[_ptr(x) for x in outs], ctypes.byref(e) if want else None,
                                        ctypes.byref(n2) if want else None))
        return e.value, n2.value

    def step_spin(self, h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta, eps=1e-3, active=None, tile=-1,
                  return_ru=False, flags=0, precision="fp64", moduli=0, sigma=None):
        """One Euler step of Eq. (9) for a state of any S_z on device copies; a dict
        with the new d1a, d1b, d2aa, d2bb, d2ab, the energy after the step and
        ||R||^2 before it (and R, U blocks with return_ru)."""
        prob, t = self.problem_spin(h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta)
        r = prob.r
        outs = [None] * 6
        if return_ru:
            outs = [torch.empty((r, r, r, r), dtype=torch.float64, device=self.device) for _ in range(6)]
        E, n2 = self.step_spin_raw(prob, eps, self.options(precision, active, tile, flags, sigma, moduli), outs)
        res = dict(d1a=t[2], d1b=t[3], d2aa=t[4], d2bb=t[5], d2ab=t[6], energy=E, norm2=n2)
        if return_ru:
            res.update(zip(("R_aa", "R_bb", "R_ab", "U_aa", "U_bb", "U_ab"), outs))
        return res

    def solve_spin_raw(self, prob, opts, sopts, capacity=256):
        """acse_solve_spin on a prepared problem; returns (SolveResult, [Trial])."""
        _check_opts(opts, prob.r, spin=True)
        res = SolveResult()
        hist = (Trial * max(1, capacity))()
        self._check(_lib.acse_solve_spin(self._h, ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(sopts),
                                         ctypes.byref(res), hist, int(capacity)))
        return res, [hist[i] for i in range(min(res.trials, capacity))]

    def solve_spin(self, h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta, eps=1e-3, de_tol=1e-6,
                   max_iter=100, control="fixed", max_halvings=8, precision="fp64", active=None, tile=-1,
                   flags=0, capacity=256, moduli=0, sigma=None, eps_max=0.0):
        """The Euler iteration of ``solve`` for a state of any S_z on device
        copies of the inputs (acse_solve_spin; controls "fixed", "backtrack"
        and "quadratic").  Returns a dict with the final d1a, d1b, d2aa, d2bb,
        d2ab (device) and the fields of ``solve``."""
        prob, t = self.problem_spin(h, V, d1a, d1b, d2aa, d2bb, d2ab, n_alpha, n_beta)
        so = SolveOptions(float(eps), float(de_tol), float(eps_max), int(max_iter),
                          CONTROLS[control] if isinstance(control, str) else int(control), int(max_halvings), 0)
        res, hist = self.solve_spin_raw(prob, self.options(precision, active, tile, flags, sigma, moduli), so,
                                        capacity)
        return dict(d1a=t[2], d1b=t[3], d2aa=t[4], d2bb=t[5], d2ab=t[6], energy0=res.energy0,
                    norm2_0=res.norm2_0, energy=res.energy, norm2=res.norm2, eps=res.eps,
                    iterations=res.iterations, trial_count=res.trials, maps=res.maps, stop=STOP_REASONS[res.stop],
                    trials=[(q.eps, q.energy, q.norm2, q.step, bool(q.accepted)) for q in hist])

    def energy_spin(self, h, V, d2aa, d2bb, d2ab, n_alpha, n_beta):
        """E = Tr(K 2D) for a state of any S_z."""
        r = _shape(h)[0]
        z = torch.zeros(r, r, dtype=torch.float64)
        prob, keep = self.problem_spin(h, V, z, z, d2aa, d2bb, d2ab, n_alpha, n_beta)
        e = ctypes.c_double(0.0)
        self._check(_lib.acse_energy_spin(self._h, ctypes.byref(prob), ctypes.byref(e)))
        return e.value

    def residual_vjp_raw(self, prob, opts, Rbar_aa, Rbar_ab, h_bar, V_bar, d1_bar, d2aa_bar, d2ab_bar):
        _check_opts(opts, prob.r)
        r = prob.r
        for name, t in (("Rbar_aa", Rbar_aa), ("Rbar_ab", Rbar_ab), ("V_bar", V_bar), ("d2aa_bar", d2aa_bar),
                        ("d2ab_bar", d2ab_bar)):
            _check_dev4(t, r, name, self.device)
        for name, t in (("h_bar", h_bar), ("d1_bar", d1_bar)):
            _check_dev2(t, r, name, self.device)
        self._check(_lib.acse_residual_vjp(self._h, ctypes.byref(prob), ctypes.byref(opts),
                                           _ptr(Rbar_aa), _ptr(Rbar_ab), _ptr(h_bar), _ptr(V_bar),
                                           _ptr(d1_bar), _ptr(d2aa_bar), _ptr(d2ab_bar)))

    def residual_vjp(self, h, V, d1, d2aa, d2ab, n_alpha, Rbar_aa, Rbar_ab, precision="fp64", tile=-1,
                     flags=0, sigma=None, moduli=0):
        """Cotangents (h, V, d1, d2aa, d2ab) of <Rbar, R> for the residual of Eq. (4),
        projected onto the symmetry subspace of each input; ``sigma`` as for
        ``options`` (the NY residual's adjoint)."""
        prob, keep = self.problem(h, V, d1, d2aa, d2ab, n_alpha)
        for name, x in (("Rbar_aa", Rbar_aa), ("Rbar_ab", Rbar_ab)):
            if _numel(x) != prob.r ** 4:
                raise ValueError(f"{name} must hold r^4 = {prob.r ** 4} elements, got shape {_shape(x)}")
        rb = [_dev(x, self.device) for x in (Rbar_aa, Rbar_ab)]
        out = [torch.empty_like(x) for x in keep]
        self.residual_vjp_raw(prob, self.options(precision, None, tile, flags, sigma, moduli), *rb, *out)
        return tuple(out)

    def residual_batched_raw(self, probs, opts, R_aa, R_ab, want_norm=True):
        """probs: sequence of Problem; R_aa/R_ab: sequences of device tensors.
        Returns the list of ||R_i||^2 (or None)."""
        n = len(probs)
        if len(R_aa) != n or len(R_ab) != n:
            raise ValueError("one R_aa and one R_ab array per instance")
        for q, prob in enumerate(probs):
            _check_opts(opts, prob.r)
            _check_dev4(R_aa[q], prob.r, f"R_aa[{q}]", self.device)
            _check_dev4(R_ab[q], prob.r, f"R_ab[{q}]", self.device)
        parr = (Problem * n)(*probs)
        ra = (ctypes.c_void_p * n)(*[t.data_ptr() for t in R_aa])
        rb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in R_ab])
        n2 = (ctypes.c_double * n)()
        self._check(_lib.acse_residual_batched(self._h, n, parr, ctypes.byref(opts), ra, rb,
                                               n2 if want_norm else None))
        return list(n2) if want_norm else None

    def autotune_batched_raw(self, probs, opts):
        for prob in probs:
            _check_opts(opts, prob.r)
        n = len(probs)
        parr = (Problem * n)(*probs)
        best = ctypes.c_int32(-1)
        times = (ctypes.c_double * NUM_TILE_CONFIGS)()
        self._check(_lib.acse_autotune_batched(self._h, n, parr, ctypes.byref(opts), ctypes.byref(best),
                                               times))
        return best.value, list(times)

    def residual_batched(self, instances, precision="fp64", tile=-1, flags=0, ny=False):
        """instances: sequence of dicts with h, V, gamma, d2aa, d2ab, N.  One
        batched call; returns [(R_aa, R_ab, norm2)] in input order.  ny=True
        selects the Nakatsuji-Yasuda 3-RDM with each instance's orbitals below
        N/2 occupied."""
        probs, keep, outs = [], [], []
        for p in instances:
            prob, t = self.problem(p["h"], p["V"], p["gamma"], p["d2aa"], p["d2ab"], p["N"] // 2)
            probs.append(prob)
            keep.append(t)
            r = prob.r
            outs.append([torch.empty((r, r, r, r), dtype=torch.float64, device=self.device)
                         for _ in range(2)])
        n2 = self.residual_batched_raw(probs, self.options(precision, None, tile, flags, True if ny else None),
                                       [o[0] for o in outs], [o[1] for o in outs])
        return [(o[0], o[1], v) for o, v in zip(outs, n2)]

    def energy_vjp_raw(self, prob, Ebar, h_bar, V_bar, d2aa_bar, d2ab_bar):
        for name, t in (("V_bar", V_bar), ("d2aa_bar", d2aa_bar), ("d2ab_bar", d2ab_bar)):
            _check_dev4(t, prob.r, name, self.device)
        _check_dev2(h_bar, prob.r, "h_bar", self.device)
        self._check(_lib.acse_energy_vjp(self._h, ctypes.byref(prob), float(Ebar), _ptr(h_bar),
                                         _ptr(V_bar), _ptr(d2aa_bar), _ptr(d2ab_bar)))

    def energy_vjp(self, h, V, d2aa, d2ab, n_alpha, Ebar=1.0):
        """Cotangents (h, V, d2aa, d2ab) of Ebar * E, E = Tr(K 2D), projected."""
        r = h.shape[0]
        prob, keep = self.problem(h, V, torch.zeros(r, r), d2aa, d2ab, n_alpha)
        out = [torch.empty_like(keep[q]) for q in (0, 1, 3, 4)]
        self.energy_vjp_raw(prob, Ebar, *out)
        return tuple(out)


class ACSEResidual(torch.autograd.Function):
    """R = F(K) of Eq. (4) as an autograd function with the hand-written adjoint.

    ``ACSEResidual.apply(ctx, h, V, d1, d2aa, d2ab, n_alpha, precision, sigma)``
    returns (R_aa, R_ab); ``sigma`` (None: Valdemoro) as for ``Context.options``.  The gradients are those of the loss restricted to the
    symmetric inputs: each is projected onto its input's symmetry subspace
    (h, d1 symmetric; V with the 8-fold symmetry of (pq|rs); d2aa antisymmetric
    within each pair and Hermitian; d2ab Hermitian and pair-exchange symmetric).
    """

    @staticmethod
    def forward(fctx, ctx, h, V, d1, d2aa, d2ab, n_alpha, precision="fp64", sigma=None):
        R_aa, R_ab, _ = ctx.residual(h, V, d1, d2aa, d2ab, n_alpha, precision, sigma=sigma)
        fctx.acse = (ctx, n_alpha, precision, sigma)
        fctx.save_for_backward(h, V, d1, d2aa, d2ab)
        return R_aa, R_ab

    @staticmethod
    def backward(fctx, Rb_aa, Rb_ab):
        ctx, n_alpha, precision, sigma = fctx.acse
        h, V, d1, d2aa, d2ab = fctx.saved_tensors
        r = h.shape[0]
        zero = torch.zeros((r, r, r, r), dtype=torch.float64, device=ctx.device)
        Rb_aa = zero if Rb_aa is None else Rb_aa
        Rb_ab = zero if Rb_ab is None else Rb_ab
        g = ctx.residual_vjp(h, V, d1, d2aa, d2ab, n_alpha, Rb_aa, Rb_ab, precision, sigma=sigma)
        return (None,) + tuple(x.to(t.dtype) for x, t in zip(g, (h, V, d1, d2aa, d2ab))) + (None, None, None)


class ACSEEnergy(torch.autograd.Function):
    """E = Tr(K 2D) (Eq. (2), Eq. (6)) with its adjoint; gradients projected as in
    ``ACSEResidual``.  ``ACSEEnergy.apply(ctx, h, V, d2aa, d2ab, n_alpha)``."""

    @staticmethod
    def forward(fctx, ctx, h, V, d2aa, d2ab, n_alpha):
        E = ctx.energy(h, V, d2aa, d2ab, n_alpha)
        fctx.acse = (ctx, n_alpha)
        fctx.save_for_backward(h, V, d2aa, d2ab)
        return torch.tensor(E, dtype=torch.float64, device=ctx.device)

    @staticmethod
    def backward(fctx, Eb):
        ctx, n_alpha = fctx.acse
        h, V, d2aa, d2ab = fctx.saved_tensors
        g = ctx.energy_vjp(h, V, d2aa, d2ab, n_alpha, float(Eb))
        return (None,) + tuple(x.to(t.dtype) for x, t in zip(g, (h, V, d2aa, d2ab))) + (None,)


# Options of ``Context.solve`` that change the iteration a checkpoint continues,
# with their defaults there.
_SOLVE_TAG_DEFAULTS = dict(de_tol=1e-6, control="fixed", max_halvings=8, eps_max=0.0, precision="fp64",
                           active=None, sigma=None, moduli=0)


def checkpoint_tag(h, V, n_alpha, **kw):
    """Hash naming the problem and the iteration of a ``solve_checkpointed`` file:
    h, V, n_alpha, the reconstruction (``sigma``), the precision of the
    contractions and its modulus count, the active mask, the step control,
    max_halvings, eps_max and de_tol (defaults as in ``Context.solve``).  The first step size is not part
    of it: a resumed run continues with the step size the file holds."""
    import hashlib
    import numpy as np

    tag = hashlib.sha256()
    for x in (h, V):
        tag.update(np.ascontiguousarray(_host64(x)).tobytes())
    tag.update(str(int(n_alpha)).encode())
    opt = {k: kw.get(k, d) for k, d in _SOLVE_TAG_DEFAULTS.items()}
    sigma = opt["sigma"]
    if sigma is not None and sigma is not False:
        tag.update(b"NY:" + (b"default" if sigma is True else bytes(str([int(x) for x in sigma]), "ascii")))
    control = opt["control"]
    control = CONTROLS[control] if isinstance(control, str) else int(control)
    precision = opt["precision"]
    precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    active = None if opt["active"] is None else [bool(a) for a in opt["active"]]
    tag.update(repr((precision, active, control, int(opt["max_halvings"]), float(opt["eps_max"]).hex(),
                     float(opt["de_tol"]).hex(), int(opt["moduli"]))).encode())
    return tag.hexdigest()


def _host64(x):
    import numpy as np
    if isinstance(x, torch.Tensor):
        return x.detach().to("cpu", torch.float64).numpy()
    return np.asarray(x, dtype=np.float64)


def trajectory(result):
    """The trajectory the method section plots, from a ``solve`` result: a
    list of (lambda, E, log10 ||R||) for the input state and each accepted step,
    lambda being the sum of the accepted step sizes (eps n at a fixed eps)."""
    import math
    out = [(0.0, result["energy0"], 0.5 * math.log10(result["norm2_0"]) if result["norm2_0"] > 0 else -math.inf)]
    lam = 0.0
    for eps, e, n2, _step, accepted in result["trials"]:
        if accepted:
            lam += eps
            out.append((lam, e, 0.5 * math.log10(n2) if n2 > 0 else -math.inf))
    return out


NOALLOC_MAX_R = 16


def residual_noalloc_raw(prob, opts, R_aa, R_ab, norm2_dev=None, stream=None):
    """acse_residual_noalloc on device arrays: no context, no allocation in the
    library (its workspace is a fixed device array for r <= 16).  The work is
    ordered on ``stream`` (torch stream; default: the current one) of the
    current device; ``norm2_dev`` (a one-element float64 device tensor) receives
    ||R||^2 if given.  Nothing is synchronised."""
    _check_opts(opts, prob.r)
    dev = R_aa.device if isinstance(R_aa, torch.Tensor) else None
    for name, t in (("R_aa", R_aa), ("R_ab", R_ab)):
        _check_dev4(t, prob.r, name, dev)
    if norm2_dev is not None and (not isinstance(norm2_dev, torch.Tensor) or norm2_dev.dtype != torch.float64
                                  or norm2_dev.device != dev or norm2_dev.numel() < 1):
        raise ValueError(f"norm2_dev must be a float64 tensor on {dev}")
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    st = _lib.acse_residual_noalloc(ctypes.c_void_p(s.cuda_stream), ctypes.byref(prob), ctypes.byref(opts),
                                    _ptr(R_aa), _ptr(R_ab), _ptr(norm2_dev))
    if st != 0:
        raise AcseError(st, _lib.acse_last_error(None).decode())


def residual_noalloc(h, V, d1, d2aa, d2ab, n_alpha, precision="fp64", device=0, stream=None):
    """R_aa, R_ab (device) and ||R||^2 through acse_residual_noalloc (r <= 16).
    The inputs and outputs are allocated here by torch; the library allocates
    nothing.  Synchronises the stream the work is ordered on before returning."""
    r = check_problem_shapes(h, V, d1, d2aa, d2ab)
    dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
    t = [_dev(x, dev) for x in (h, V, d1, d2aa, d2ab)]
    prob = Problem(r, int(n_alpha), int(n_alpha), *[x.data_ptr() for x in t])
    R_aa = torch.empty((r, r, r, r), dtype=torch.float64, device=dev)
    R_ab = torch.empty_like(R_aa)
    n2 = torch.empty(1, dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        residual_noalloc_raw(prob, Context.options(precision), R_aa, R_ab, n2, s)
        # the work is ordered on s: wait for it before the norm is read and the
        # input copies made here are released
        s.synchronize()
        return R_aa, R_ab, float(n2.item())


def status_str(code):
    return _lib.acse_status_str(int(code)).decode()


_contexts = {}


def context(r, device=0):
    """A cached context with room for r (grown as needed)."""
    key = device
    c = _contexts.get(key)
    if c is None or c.r_max < r:
        if c is not None:
            c.close()
        c = Context(max(r, 8), device)
        _contexts[key] = c
    return c


def residual(h, V, d1, d2aa, d2ab, n_alpha, precision="fp64"):
    return context(h.shape[0]).residual(h, V, d1, d2aa, d2ab, n_alpha, precision)


def energy(h, V, d2aa, d2ab, n_alpha):
    return context(h.shape[0]).energy(h, V, d2aa, d2ab, n_alpha)


def step(h, V, d1, d2aa, d2ab, n_alpha, eps=1e-3, precision="fp64", active=None):
    return context(h.shape[0]).step(h, V, d1, d2aa, d2ab, n_alpha, eps, precision, active)
