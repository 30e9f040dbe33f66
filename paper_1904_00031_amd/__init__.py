"""Python binding of libnqs (argument marshalling only).

Every function here checks shapes, dtypes and devices of torch tensors, then calls the C
ABI declared in ``include/nqs.h`` with raw device pointers and the current HIP stream.
All arithmetic of the VMC hot path runs in the library's HIP kernels. There is no CPU
fallback: if ``libnqs.so`` is missing, :func:`load` raises.

Names follow the C ABI (``nqs_sample``, ``nqs_local_energy``, ...); :class:`Model`
offers the same calls as methods.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnqs.so")

F64, F32, BF16 = 0, 1, 2
TIME_NONE, TIME_SWEEP, TIME_SV, TIME_ELOC = 0, 1, 2, 3
TFIM, HEISENBERG = 0, 1
MOVE_FLIP, MOVE_EXCHANGE = 0, 1
ACT_LNCOSH, ACT_TANH = 0, 1
OK, ENOTCONV, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5

_lib = None


class NQSError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.nqs_status_string(status).decode() if _lib is not None else str(status)
        super().__init__("%s: %s (status %d)" % (where, msg, status))


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
        ("is_complex", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("n_bonds", ctypes.c_int32 * 2), ("bonds", ctypes.c_void_p * 2),
        ("ham", ctypes.c_int32), ("J", ctypes.c_double * 2), ("h", ctypes.c_double),
        ("marshall", ctypes.c_int32), ("sublattice", ctypes.c_void_p), ("move", ctypes.c_int32),
        ("n_symm", ctypes.c_int32), ("symm", ctypes.c_void_p),
        ("n_layers", ctypes.c_int32), ("layer_sizes", ctypes.c_void_p),
        ("activations", ctypes.c_void_p),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("n_candidates", ctypes.c_int32), ("chosen", ctypes.c_int32),
        ("pairs", ctypes.c_int32 * 4), ("us", ctypes.c_double * 4),
    ]

    def as_dict(self):
        n = self.n_candidates
        return {"chosen": self.chosen, "pairs": list(self.pairs[:n]), "us": list(self.us[:n])}


class SRInfo(ctypes.Structure):
    _fields_ = [
        ("cg_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("cg_resid", ctypes.c_double), ("energy_re", ctypes.c_double),
        ("energy_im", ctypes.c_double), ("variance", ctypes.c_double),
        ("force_norm", ctypes.c_double), ("energy_err", ctypes.c_double),
        ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


SR_INFO_BYTES = ctypes.sizeof(SRInfo)


class OverlapInfo(ctypes.Structure):
    _fields_ = [
        ("loss", ctypes.c_double), ("overlap", ctypes.c_double), ("grad_norm", ctypes.c_double),
        ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def sr_infos_from_device(buf, count=1):
    """Decode nqs_sr_info structs written to a device uint8 tensor by the stream-ordered
    SR calls (copies the bytes to the host; synchronises)."""
    raw = bytes(buf[:count * SR_INFO_BYTES].cpu().numpy().tobytes())
    return [SRInfo.from_buffer_copy(raw, k * SR_INFO_BYTES).as_dict() for k in range(count)]


def load(path=LIB_PATH):
    """Load libnqs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libnqs.so not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "nqs_status_string": (ctypes.c_char_p, [i32]),
        "nqs_hypercube": (i32, [i32, i32, i32, vp, vp, vp, vp]),
        "nqs_hypercube_translations": (i32, [i32, i32, vp]),
        "nqs_model_create": (i32, [ctypes.POINTER(_Desc), ctypes.POINTER(vp)]),
        "nqs_model_destroy": (None, [vp]),
        "nqs_n_params": (i64, [vp]),
        "nqs_chain_init": (i32, [vp, vp, i32, u64, i32, vp]),
        "nqs_sample": (i32, [vp, vp, vp, i32, i32, i32, u64, u64, i32, vp, vp, vp, vp]),
        "nqs_sample_pt": (i32, [vp, vp, vp, vp, i32, i32, i32, i32, u64, u64, i32, vp, vp, vp, vp,
                                vp]),
        "nqs_log_psi": (i32, [vp, vp, vp, i64, vp, vp]),
        "nqs_local_energy": (i32, [vp, vp, vp, i64, vp, vp]),
        "nqs_log_psi_grad": (i32, [vp, vp, vp, i64, vp, vp, vp, vp, vp]),
        "nqs_target_cdf": (i32, [vp, vp, i64, vp, vp]),
        "nqs_target_draw": (i32, [vp, vp, i64, vp, vp, i64, u64, u64, vp, vp, vp, vp]),
        "nqs_overlap_step": (i32, [vp, vp, vp, vp, i64, ctypes.c_double, vp, vp]),
        "nqs_log_psi_grad_noalloc": (i32, [vp, vp, vp, i64, vp, vp, vp, vp, vp]),
        "nqs_sr_workspace_bytes": (ctypes.c_size_t, [vp, i64]),
        "nqs_sr_step": (i32, [vp, vp, vp, vp, i64, i32, f64, f64, f64, i32, vp, ctypes.c_size_t,
                              ctypes.POINTER(SRInfo), vp]),
        "nqs_sr_step_async": (i32, [vp, vp, vp, vp, i64, i32, f64, f64, f64, i32, vp,
                                    ctypes.c_size_t, vp, vp]),
        "nqs_sr_prepare": (i32, [vp, vp, vp, i64, vp, ctypes.c_size_t, vp]),
        "nqs_sr_matvec": (i32, [vp, vp, i64, vp, ctypes.c_size_t, vp, f64, vp, vp]),
        "nqs_set_sv_shape": (i32, [vp, i32]),
        "nqs_set_cg_graphs": (i32, [vp, i32]),
        "nqs_time_kernel": (i32, [vp, i32]),
        "nqs_kernel_ms": (i32, [vp, ctypes.POINTER(ctypes.c_float)]),
        "nqs_kernel_times": (i32, [vp, ctypes.POINTER(ctypes.c_float), i32,
                                   ctypes.POINTER(ctypes.c_int32)]),
        "nqs_batch_create": (i32, [ctypes.POINTER(_Desc), i32, ctypes.POINTER(vp)]),
        "nqs_batch_destroy": (None, [vp]),
        "nqs_batch_n_params": (i64, [vp, i32]),
        "nqs_batch_chain_init": (i32, [vp, vp, ctypes.POINTER(i32), u64, vp]),
        "nqs_batch_sample": (i32, [vp, vp, vp, ctypes.POINTER(i32), i32, i32, u64, u64, vp, vp,
                                   vp, vp, vp]),
        "nqs_batch_sr_workspace_bytes": (ctypes.c_size_t, [vp, ctypes.POINTER(i64)]),
        "nqs_batch_sr_step": (i32, [vp, vp, vp, vp, ctypes.POINTER(i64), vp, f64, f64, f64, i32,
                                    vp, ctypes.c_size_t, ctypes.POINTER(SRInfo), vp]),
        "nqs_batch_sr_step_async": (i32, [vp, vp, vp, vp, ctypes.POINTER(i64), vp, f64, f64, f64,
                                          i32, vp, ctypes.c_size_t, vp, vp]),
        "nqs_autotune": (i32, [vp, vp, vp, i64, vp, ctypes.c_size_t, ctypes.POINTER(TuneReport), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["nqs_status_string", "nqs_hypercube", "nqs_hypercube_translations",
            "nqs_model_create", "nqs_model_destroy",
            "nqs_n_params", "nqs_chain_init", "nqs_sample", "nqs_sample_pt", "nqs_log_psi",
            "nqs_local_energy",
            "nqs_log_psi_grad", "nqs_log_psi_grad_noalloc", "nqs_sr_workspace_bytes", "nqs_sr_step", "nqs_sr_step_async",
            "nqs_sr_prepare",
            "nqs_sr_matvec", "nqs_autotune", "nqs_set_sv_shape", "nqs_set_cg_graphs",
            "nqs_time_kernel", "nqs_kernel_ms", "nqs_kernel_times",
            "nqs_target_cdf", "nqs_target_draw", "nqs_overlap_step",
            "nqs_batch_create",
            "nqs_batch_destroy", "nqs_batch_n_params", "nqs_batch_chain_init",
            "nqs_batch_sample", "nqs_batch_sr_workspace_bytes", "nqs_batch_sr_step",
            "nqs_batch_sr_step_async"]


def _check(status, where, allow=(OK,)):
    if status not in allow:
        raise NQSError(status, where)
    return status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, dtype, shape=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def nqs_hypercube(L, ndim, with_diagonals=False):
    """Bond lists (color 0, color 1) and sublattice parity of a periodic L^ndim lattice."""
    load()
    n = L ** ndim
    b0 = np.zeros((max(1, ndim * n), 2), dtype=np.int32)
    b1 = np.zeros((max(1, 2 * n), 2), dtype=np.int32)
    sub = np.zeros(n, dtype=np.int8)
    nb = np.zeros(2, dtype=np.int32)
    _check(_lib.nqs_hypercube(L, ndim, int(bool(with_diagonals)), b0.ctypes.data, b1.ctypes.data,
                              sub.ctypes.data, nb.ctypes.data), "nqs_hypercube")
    return [b0[:nb[0]].copy(), b1[:nb[1]].copy()], sub


def nqs_hypercube_translations(L, ndim):
    """The L^ndim translations of the periodic hypercube as site permutations [G, N]."""
    load()
    n = L ** ndim
    perm = np.zeros((n, n), dtype=np.int32)
    _check(_lib.nqs_hypercube_translations(L, ndim, perm.ctypes.data), "nqs_hypercube_translations")
    return perm


def _fill_desc(d, n_sites, n_hidden, bonds, ham, J, h, marshall, sub, move, is_complex, prec,
               symm=None, layers=None, acts=None):
    """Fill an nqs_model_desc; bonds (two int32 [B, 2] arrays), sub and symm (int32 [G, N])
    must stay alive."""
    d.n_sites, d.n_hidden = int(n_sites), int(n_hidden)
    d.is_complex, d.prec = int(bool(is_complex)), int(prec)
    for c in range(2):
        d.n_bonds[c] = bonds[c].shape[0]
        d.bonds[c] = bonds[c].ctypes.data if bonds[c].shape[0] else None
    d.ham = int(ham)
    d.J[0], d.J[1] = float(J[0]), float(J[1])
    d.h = float(h)
    d.marshall = int(bool(marshall))
    d.sublattice = sub.ctypes.data if sub is not None else None
    d.move = int(move)
    d.n_symm = 0 if symm is None else int(symm.shape[0])
    d.symm = symm.ctypes.data if symm is not None else None
    d.n_layers = 0 if layers is None else int(layers.shape[0])
    d.layer_sizes = layers.ctypes.data if layers is not None else None
    d.activations = acts.ctypes.data if acts is not None else None


class Model:
    """Handle of one lattice model + RBM shape + compute precision (nqs_model_create)."""

    def __init__(self, n_sites, n_hidden, bonds, ham=TFIM, J=(1.0, 0.0), h=1.0, marshall=False,
                 sublattice=None, move=MOVE_FLIP, is_complex=False, prec=F64, symm=None,
                 layers=None, activations=None):
        """symm: site permutations [G, N] of a symmetric RBM (n_hidden = alpha G), or None.
        layers / activations: widths and ACT_* codes of a feed-forward network (n_hidden is
        then ignored), or None for an RBM."""
        load()
        self.n_sites, self.n_hidden = int(n_sites), int(n_hidden)
        self.is_complex, self.prec = bool(is_complex), int(prec)
        self.ham, self.move = int(ham), int(move)
        self._bonds = [np.ascontiguousarray(np.asarray(b, dtype=np.int32).reshape(-1, 2)) for b in bonds]
        while len(self._bonds) < 2:
            self._bonds.append(np.zeros((0, 2), dtype=np.int32))
        self._sub = None if sublattice is None else np.ascontiguousarray(np.asarray(sublattice, dtype=np.int8))
        self._symm = None if symm is None else np.ascontiguousarray(np.asarray(symm, dtype=np.int32))
        self.n_symm = 0 if symm is None else int(self._symm.shape[0])
        self._layers = None if layers is None else np.ascontiguousarray(np.asarray(layers, dtype=np.int32))
        self._acts = None
        if layers is not None:
            acts = [ACT_LNCOSH] * len(layers) if activations is None else activations
            self._acts = np.ascontiguousarray(np.asarray(acts, dtype=np.int32))
            self.n_hidden = int(self._layers[0])
        self.layers = None if layers is None else [int(x) for x in self._layers]
        d = _Desc()
        _fill_desc(d, self.n_sites, self.n_hidden, self._bonds, self.ham, J, h, marshall,
                   self._sub, self.move, self.is_complex, self.prec, self._symm, self._layers,
                   self._acts)
        h_ = ctypes.c_void_p()
        _check(_lib.nqs_model_create(ctypes.byref(d), ctypes.byref(h_)), "nqs_model_create")
        self._h = h_
        self.n_params = int(_lib.nqs_n_params(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nqs_model_destroy(self._h)
            self._h = None

    # dtypes ---------------------------------------------------------------------------
    @property
    def param_dtype(self):
        import torch
        if self.prec == F64:
            return torch.complex128 if self.is_complex else torch.float64
        return torch.complex64 if self.is_complex else torch.float32

    @property
    def value_dtype(self):
        import torch
        return torch.complex128 if self.is_complex else torch.float64

    # calls ----------------------------------------------------------------------------
    def chain_init(self, chain_sigma, seed, chain_offset=0):
        import torch
        _need(chain_sigma, "chain_sigma", torch.int8)
        C = chain_sigma.shape[0]
        _need(chain_sigma, "chain_sigma", torch.int8, (C, self.n_sites))
        _check(_lib.nqs_chain_init(self._h, _ptr(chain_sigma), C, seed, chain_offset, _stream()),
               "nqs_chain_init")
        return chain_sigma

    def sample(self, params, chain_sigma, n_sweeps, n_discard, seed, counter, chain_offset=0,
               samples=None, n_accepted=None, eloc=None, with_eloc=False):
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        C = chain_sigma.shape[0]
        _need(chain_sigma, "chain_sigma", torch.int8, (C, self.n_sites))
        dev = chain_sigma.device
        if samples is None:
            samples = torch.empty((n_sweeps, C, self.n_sites), dtype=torch.int8, device=dev)
        _need(samples, "samples", torch.int8, (n_sweeps, C, self.n_sites))
        if n_accepted is not None:
            _need(n_accepted, "n_accepted", torch.int64, (C,))
        if with_eloc and eloc is None:
            eloc = torch.empty(n_sweeps * C, dtype=self.value_dtype, device=dev)
        if eloc is not None:
            _need(eloc, "eloc", self.value_dtype, (n_sweeps * C,))
        _check(_lib.nqs_sample(self._h, _ptr(params), _ptr(chain_sigma), C, n_sweeps, n_discard,
                               seed, counter, chain_offset, _ptr(samples), _ptr(n_accepted),
                               _ptr(eloc), _stream()), "nqs_sample")
        return samples, eloc

    def sample_pt(self, params, replicas, temp_index, n_sweeps, n_discard, seed, counter,
                  chain_offset=0, samples=None, n_accepted=None, n_swaps=None, eloc=None,
                  with_eloc=False):
        """Parallel tempering: replicas [C, R, N] int8 and temp_index [C, R] int32 (both
        updated in place); returns (samples [S, C, N], eloc)."""
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        C, R = replicas.shape[0], replicas.shape[1]
        _need(replicas, "replicas", torch.int8, (C, R, self.n_sites))
        _need(temp_index, "temp_index", torch.int32, (C, R))
        dev = replicas.device
        if samples is None:
            samples = torch.empty((n_sweeps, C, self.n_sites), dtype=torch.int8, device=dev)
        _need(samples, "samples", torch.int8, (n_sweeps, C, self.n_sites))
        if n_accepted is not None:
            _need(n_accepted, "n_accepted", torch.int64, (C * R,))
        if n_swaps is not None:
            _need(n_swaps, "n_swaps", torch.int64, (C,))
        if with_eloc and eloc is None:
            eloc = torch.empty(n_sweeps * C, dtype=self.value_dtype, device=dev)
        if eloc is not None:
            _need(eloc, "eloc", self.value_dtype, (n_sweeps * C,))
        _check(_lib.nqs_sample_pt(self._h, _ptr(params), _ptr(replicas), _ptr(temp_index), C, R,
                                  n_sweeps, n_discard, seed, counter, chain_offset, _ptr(samples),
                                  _ptr(n_accepted), _ptr(n_swaps), _ptr(eloc), _stream()),
               "nqs_sample_pt")
        return samples, eloc

    def log_psi(self, params, sigma, out=None):
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        if out is None:
            out = torch.empty(n, dtype=self.value_dtype, device=sigma.device)
        _need(out, "logpsi", self.value_dtype, (n,))
        _check(_lib.nqs_log_psi(self._h, _ptr(params), _ptr(sigma), n, _ptr(out), _stream()),
               "nqs_log_psi")
        return out

    def local_energy(self, params, sigma, out=None):
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        if out is None:
            out = torch.empty(n, dtype=self.value_dtype, device=sigma.device)
        _need(out, "eloc", self.value_dtype, (n,))
        _check(_lib.nqs_local_energy(self._h, _ptr(params), _ptr(sigma), n, _ptr(out), _stream()),
               "nqs_local_energy")
        return out

    def log_psi_grad(self, params, sigma, u=None, v=None, vjp=None, jvp=None, noalloc=False):
        """vjp = O^dagger u (length P), jvp = O v (length n). noalloc: through
        nqs_log_psi_grad_noalloc (the library's fixed per-device scratch, no allocation);
        outputs must then be given."""
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        if noalloc and ((u is not None and vjp is None) or (v is not None and jvp is None)):
            raise ValueError("noalloc: pass the output tensors (vjp, jvp)")
        if u is not None:
            _need(u, "u", self.value_dtype, (n,))
            if vjp is None:
                vjp = torch.empty(self.n_params, dtype=self.value_dtype, device=sigma.device)
            _need(vjp, "vjp", self.value_dtype, (self.n_params,))
        if v is not None:
            _need(v, "v", self.value_dtype, (self.n_params,))
            if jvp is None:
                jvp = torch.empty(n, dtype=self.value_dtype, device=sigma.device)
            _need(jvp, "jvp", self.value_dtype, (n,))
        fn = _lib.nqs_log_psi_grad_noalloc if noalloc else _lib.nqs_log_psi_grad
        _check(fn(self._h, _ptr(params), _ptr(sigma), n,
                  _ptr(u) if u is not None else None,
                  _ptr(vjp) if u is not None else None,
                  _ptr(v) if v is not None else None,
                  _ptr(jvp) if v is not None else None, _stream()),
               "nqs_log_psi_grad_noalloc" if noalloc else "nqs_log_psi_grad")
        return vjp, jvp

    def sr_workspace_bytes(self, n):
        return int(_lib.nqs_sr_workspace_bytes(self._h, n))

    def _sr_args(self, params, sigma, eloc, workspace):
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        _need(eloc, "eloc", self.value_dtype, (n,))
        nbytes = self.sr_workspace_bytes(n)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=sigma.device)
        _need(workspace, "workspace", torch.uint8)
        return n, workspace

    def sr_step(self, params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter, workspace=None,
                n_chains=0):
        """One SR update of params in place; returns the info dict (cg_iters, energy,
        energy_err, status, ...). n_chains: samples laid out [sweeps, n_chains] for the
        energy error bar (0: every sample its own chain)."""
        n, workspace = self._sr_args(params, sigma, eloc, workspace)
        info = SRInfo()
        st = _lib.nqs_sr_step(self._h, _ptr(params), _ptr(sigma), _ptr(eloc), n, int(n_chains),
                              float(lr), float(diag_shift), float(cg_tol), int(cg_maxiter),
                              _ptr(workspace), workspace.numel(), ctypes.byref(info), _stream())
        _check(st, "nqs_sr_step", allow=(OK, ENOTCONV, ENONFINITE))
        return info.as_dict()

    def sr_step_async(self, params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter,
                      workspace=None, n_chains=0, info=None):
        """Stream-ordered SR update (cg_maxiter iteration slots, nothing read back). info: a
        device uint8 tensor of at least SR_INFO_BYTES that receives the nqs_sr_info; returns
        it (decode with sr_infos_from_device)."""
        import torch
        n, workspace = self._sr_args(params, sigma, eloc, workspace)
        if info is None:
            info = torch.zeros(SR_INFO_BYTES, dtype=torch.uint8, device=sigma.device)
        _need(info, "info", torch.uint8)
        if info.numel() < SR_INFO_BYTES:
            raise ValueError("info needs %d bytes" % SR_INFO_BYTES)
        _check(_lib.nqs_sr_step_async(self._h, _ptr(params), _ptr(sigma), _ptr(eloc), n,
                                      int(n_chains), float(lr), float(diag_shift), float(cg_tol),
                                      int(cg_maxiter), _ptr(workspace), workspace.numel(),
                                      _ptr(info), _stream()), "nqs_sr_step_async")
        return info

    def target_cdf(self, log_target):
        """Cumulative |t|^2 (scaled) of a training set's log targets [n_states]."""
        import torch
        n = log_target.shape[0]
        _need(log_target, "log_target", self.value_dtype, (n,))
        cdf = torch.empty(n, dtype=torch.float64, device=log_target.device)
        _check(_lib.nqs_target_cdf(self._h, _ptr(log_target), n, _ptr(cdf), _stream()),
               "nqs_target_cdf")
        return cdf

    def target_draw(self, cdf, states, log_target, n, seed, counter):
        """n draws from |t|^2 over the training set; returns (sigma [n, N], log t [n],
        index [n])."""
        import torch
        ns = states.shape[0]
        _need(cdf, "cdf", torch.float64, (ns,))
        _need(states, "states", torch.int8, (ns, self.n_sites))
        _need(log_target, "log_target", self.value_dtype, (ns,))
        dev = states.device
        sigma = torch.empty((n, self.n_sites), dtype=torch.int8, device=dev)
        lt = torch.empty(n, dtype=self.value_dtype, device=dev)
        idx = torch.empty(n, dtype=torch.int64, device=dev)
        _check(_lib.nqs_target_draw(self._h, _ptr(cdf), ns, _ptr(states), _ptr(log_target), n,
                                    seed, counter, _ptr(sigma), _ptr(lt), _ptr(idx), _stream()),
               "nqs_target_draw")
        return sigma, lt, idx

    def overlap_step(self, params, sigma, log_target, lr):
        """One step of Eq. 2 from target-distributed samples (params updated in place);
        returns the info dict (loss, overlap, grad_norm, status)."""
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        _need(log_target, "log_target", self.value_dtype, (n,))
        info = OverlapInfo()
        _check(_lib.nqs_overlap_step(self._h, _ptr(params), _ptr(sigma), _ptr(log_target), n,
                                     float(lr), ctypes.byref(info), _stream()),
               "nqs_overlap_step", allow=(OK, ENONFINITE))
        return info.as_dict()

    def sr_prepare(self, params, sigma, workspace=None):
        """Prepare the implicit S of these samples; returns the workspace to pass to
        sr_matvec."""
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        nbytes = self.sr_workspace_bytes(n)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=sigma.device)
        _need(workspace, "workspace", torch.uint8)
        _check(_lib.nqs_sr_prepare(self._h, _ptr(params), _ptr(sigma), n, _ptr(workspace),
                                   workspace.numel(), _stream()), "nqs_sr_prepare")
        return workspace

    def sr_matvec(self, sigma, workspace, v, diag_shift=0.0, out=None):
        """out = (S + diag_shift I) v with the workspace of sr_prepare."""
        import torch
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        _need(v, "v", self.value_dtype, (self.n_params,))
        if out is None:
            out = torch.empty(self.n_params, dtype=self.value_dtype, device=sigma.device)
        _need(out, "out", self.value_dtype, (self.n_params,))
        _check(_lib.nqs_sr_matvec(self._h, _ptr(sigma), n, _ptr(workspace), workspace.numel(),
                                  _ptr(v), float(diag_shift), _ptr(out), _stream()),
               "nqs_sr_matvec")
        return out


    def autotune(self, params, sigma, workspace=None):
        """Time the S v kernel shapes for these samples and keep the fastest; returns
        {"chosen", "pairs", "us"}."""
        import torch
        _need(params, "params", self.param_dtype, (self.n_params,))
        n = sigma.shape[0]
        _need(sigma, "sigma", torch.int8, (n, self.n_sites))
        if workspace is None:
            workspace = torch.empty(self.sr_workspace_bytes(n), dtype=torch.uint8,
                                    device=sigma.device)
        _need(workspace, "workspace", torch.uint8)
        rep = TuneReport()
        _check(_lib.nqs_autotune(self._h, _ptr(params), _ptr(sigma), n, _ptr(workspace),
                                 workspace.numel(), ctypes.byref(rep), _stream()), "nqs_autotune")
        return rep.as_dict()


    def set_sv_shape(self, pairs):
        _check(_lib.nqs_set_sv_shape(self._h, int(pairs)), "nqs_set_sv_shape")

    def set_cg_graphs(self, enable):
        _check(_lib.nqs_set_cg_graphs(self._h, int(bool(enable))), "nqs_set_cg_graphs")

    def time_kernel(self, what):
        """Record HIP events around launches of one kind (TIME_SWEEP, TIME_SV, TIME_ELOC;
        TIME_NONE stops)."""
        _check(_lib.nqs_time_kernel(self._h, int(what)), "nqs_time_kernel")

    def kernel_ms(self):
        """Milliseconds between the events of the last timed launch (waits for it)."""
        ms = ctypes.c_float()
        _check(_lib.nqs_kernel_ms(self._h, ctypes.byref(ms)), "nqs_kernel_ms")
        return float(ms.value)

    def kernel_times(self):
        """The event pairs of the last timed call, one time (ms) per launch, in order."""
        buf = (ctypes.c_float * 8)()
        count = ctypes.c_int32()
        _check(_lib.nqs_kernel_times(self._h, buf, 8, ctypes.byref(count)), "nqs_kernel_times")
        return [float(buf[k]) for k in range(count.value)]


class Batch:
    """K independent models sampled together (nqs_batch_*). specs: list of dicts with the
    keyword arguments of Model (n_sites, n_hidden, bonds, ham, J, h, marshall, sublattice,
    move, is_complex, prec); all with the same is_complex and prec. Buffers are flat
    tensors holding the models' buffers back to back (see include/nqs.h)."""

    def __init__(self, specs):
        load()
        self.K = len(specs)
        arr = (_Desc * self.K)()
        self._keep = []
        self.n_sites, self.n_hidden = [], []
        for k, sp in enumerate(specs):
            sp = dict(sp)
            bonds = [np.ascontiguousarray(np.asarray(b, dtype=np.int32).reshape(-1, 2))
                     for b in sp["bonds"]]
            while len(bonds) < 2:
                bonds.append(np.zeros((0, 2), dtype=np.int32))
            sub = sp.get("sublattice")
            sub = None if sub is None else np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
            self._keep.append((bonds, sub))
            _fill_desc(arr[k], sp["n_sites"], sp["n_hidden"], bonds, sp.get("ham", TFIM),
                       sp.get("J", (1.0, 0.0)), sp.get("h", 1.0), sp.get("marshall", False), sub,
                       sp.get("move", MOVE_FLIP), sp.get("is_complex", False), sp.get("prec", F64))
            self.n_sites.append(int(sp["n_sites"]))
            self.n_hidden.append(int(sp["n_hidden"]))
        self.is_complex = bool(specs[0].get("is_complex", False))
        self.prec = int(specs[0].get("prec", F64))
        h_ = ctypes.c_void_p()
        _check(_lib.nqs_batch_create(arr, self.K, ctypes.byref(h_)), "nqs_batch_create")
        self._h = h_
        self.n_params = [int(_lib.nqs_batch_n_params(self._h, k)) for k in range(self.K)]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.nqs_batch_destroy(self._h)
            self._h = None

    param_dtype = Model.param_dtype
    value_dtype = Model.value_dtype

    def offsets(self, sizes):
        return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    def chain_init(self, chains, n_chains, seed):
        nc = (ctypes.c_int32 * self.K)(*[int(c) for c in n_chains])
        _need(chains, "chain_sigma", __import__("torch").int8,
              (sum(int(c) * n for c, n in zip(n_chains, self.n_sites)),))
        _check(_lib.nqs_batch_chain_init(self._h, _ptr(chains), nc, seed, _stream()),
               "nqs_batch_chain_init")
        return chains

    def sample(self, params, chains, n_chains, n_sweeps, n_discard, seed, counter,
               samples=None, n_accepted=None, eloc=None, with_eloc=True, counter_dev=None):
        import torch
        nc = (ctypes.c_int32 * self.K)(*[int(c) for c in n_chains])
        _need(params, "params", self.param_dtype, (sum(self.n_params),))
        spins = sum(int(c) * n for c, n in zip(n_chains, self.n_sites))
        _need(chains, "chain_sigma", torch.int8, (spins,))
        if samples is None:
            samples = torch.empty(n_sweeps * spins, dtype=torch.int8, device=chains.device)
        _need(samples, "samples", torch.int8, (n_sweeps * spins,))
        if n_accepted is not None:
            _need(n_accepted, "n_accepted", torch.int64, (sum(int(c) for c in n_chains),))
        if with_eloc and eloc is None:
            eloc = torch.empty(n_sweeps * sum(int(c) for c in n_chains), dtype=self.value_dtype,
                               device=chains.device)
        if eloc is not None:
            _need(eloc, "eloc", self.value_dtype, (n_sweeps * sum(int(c) for c in n_chains),))
        if counter_dev is not None:
            _need(counter_dev, "counter_dev", torch.int64, (1,))
        _check(_lib.nqs_batch_sample(self._h, _ptr(params), _ptr(chains), nc, n_sweeps, n_discard,
                                     seed, counter, _ptr(counter_dev), _ptr(samples),
                                     _ptr(n_accepted), _ptr(eloc), _stream()), "nqs_batch_sample")
        return samples, eloc

    def sr_workspace_bytes(self, n_samples):
        ns = (ctypes.c_int64 * self.K)(*[int(x) for x in n_samples])
        return int(_lib.nqs_batch_sr_workspace_bytes(self._h, ns))

    def _sr_args(self, params, samples, eloc, n_samples, n_chains, workspace):
        import torch
        ns = (ctypes.c_int64 * self.K)(*[int(x) for x in n_samples])
        nc = None if n_chains is None else (ctypes.c_int32 * self.K)(*[int(x) for x in n_chains])
        _need(params, "params", self.param_dtype, (sum(self.n_params),))
        _need(samples, "samples", torch.int8, (sum(int(x) * n for x, n in zip(n_samples, self.n_sites)),))
        _need(eloc, "eloc", self.value_dtype, (sum(int(x) for x in n_samples),))
        nbytes = int(_lib.nqs_batch_sr_workspace_bytes(self._h, ns))
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=samples.device)
        _need(workspace, "workspace", torch.uint8)
        return ns, nc, workspace

    def sr_step(self, params, samples, eloc, n_samples, lr, diag_shift, cg_tol, cg_maxiter,
                workspace=None, n_chains=None):
        """One SR step of every model; returns a list of info dicts."""
        ns, nc, workspace = self._sr_args(params, samples, eloc, n_samples, n_chains, workspace)
        infos = (SRInfo * self.K)()
        _check(_lib.nqs_batch_sr_step(self._h, _ptr(params), _ptr(samples), _ptr(eloc), ns,
                                      nc, float(lr), float(diag_shift), float(cg_tol),
                                      int(cg_maxiter), _ptr(workspace), workspace.numel(), infos,
                                      _stream()),
               "nqs_batch_sr_step", allow=(OK, ENOTCONV, ENONFINITE))
        return [infos[k].as_dict() for k in range(self.K)]

    def sr_step_async(self, params, samples, eloc, n_samples, lr, diag_shift, cg_tol,
                      cg_maxiter, workspace=None, n_chains=None, info=None):
        """Stream-ordered SR step of every model; info: device uint8 tensor of at least
        K * SR_INFO_BYTES receiving the K nqs_sr_info structs (returned)."""
        import torch
        ns, nc, workspace = self._sr_args(params, samples, eloc, n_samples, n_chains, workspace)
        if info is None:
            info = torch.zeros(self.K * SR_INFO_BYTES, dtype=torch.uint8, device=samples.device)
        _need(info, "info", torch.uint8)
        if info.numel() < self.K * SR_INFO_BYTES:
            raise ValueError("info needs %d bytes" % (self.K * SR_INFO_BYTES))
        _check(_lib.nqs_batch_sr_step_async(self._h, _ptr(params), _ptr(samples), _ptr(eloc), ns,
                                            nc, float(lr), float(diag_shift), float(cg_tol),
                                            int(cg_maxiter), _ptr(workspace), workspace.numel(),
                                            _ptr(info), _stream()), "nqs_batch_sr_step_async")
        return info


# C-ABI-named module functions --------------------------------------------------------
def nqs_model_create(**kw):
    return Model(**kw)


def nqs_chain_init(model, chain_sigma, seed, chain_offset=0):
    return model.chain_init(chain_sigma, seed, chain_offset)


def nqs_sample(model, params, chain_sigma, n_sweeps, n_discard, seed, counter, **kw):
    return model.sample(params, chain_sigma, n_sweeps, n_discard, seed, counter, **kw)


def nqs_log_psi(model, params, sigma, out=None):
    return model.log_psi(params, sigma, out)


def nqs_local_energy(model, params, sigma, out=None):
    return model.local_energy(params, sigma, out)


def nqs_log_psi_grad(model, params, sigma, u=None, v=None, vjp=None, jvp=None):
    return model.log_psi_grad(params, sigma, u=u, v=v, vjp=vjp, jvp=jvp)


def nqs_sr_workspace_bytes(model, n):
    return model.sr_workspace_bytes(n)


def nqs_sr_prepare(model, params, sigma, workspace=None):
    return model.sr_prepare(params, sigma, workspace)


def nqs_sr_matvec(model, sigma, workspace, v, diag_shift=0.0, out=None):
    return model.sr_matvec(sigma, workspace, v, diag_shift, out)


def nqs_set_sv_shape(model, pairs):
    return model.set_sv_shape(pairs)


def nqs_autotune(model, params, sigma, workspace=None):
    return model.autotune(params, sigma, workspace)


def nqs_sr_step(model, params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter, workspace=None,
                n_chains=0):
    return model.sr_step(params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter, workspace,
                         n_chains)


def nqs_sr_step_async(model, params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter,
                      workspace=None, n_chains=0, info=None):
    return model.sr_step_async(params, sigma, eloc, lr, diag_shift, cg_tol, cg_maxiter,
                               workspace, n_chains, info)
