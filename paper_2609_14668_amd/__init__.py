"""Python binding of libdqmc.so (include/dqmc.h): argument marshalling only.

Every step of the DQMC sweep runs in the library's HIP kernels on the GPU;
PyTorch is used here only to own the device workspace and to supply the HIP
stream.  The module-level functions carry the C names; ``Simulation`` wraps a
handle.  If the library has not been built, importing the binding raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdqmc.so")

DQMC_OK = 0
STATUS = {0: "DQMC_OK", -1: "DQMC_EINVAL", -2: "DQMC_ENOMEM", -3: "DQMC_EHIP", -4: "DQMC_ENUMERIC",
          -5: "DQMC_ESTATE", -6: "DQMC_EUNSUPPORTED"}
OBS_FIELDS = ("n", "D", "ekin", "e", "Szz_G", "Szz_dk", "m2", "Rm2", "phase_cos", "phase_sin", "chi_e", "GAB_dirac")
SERIES_FIELDS = OBS_FIELDS[:11]


class DqmcError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))


class InstanceDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("t", ctypes.c_double), ("U", ctypes.c_double),
                ("beta", ctypes.c_double), ("dtau", ctypes.c_double),
                ("theta1", ctypes.c_double), ("theta2", ctypes.c_double),
                ("n_delay", ctypes.c_int32), ("n_stab", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("sym_measure", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("channel", ctypes.c_int32)]


class Obs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in OBS_FIELDS] + [("n_meas", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("proposals", ctypes.c_int64), ("accepted", ctypes.c_int64), ("flushes", ctypes.c_int64),
                ("sweeps", ctypes.c_int64), ("drift_max", ctypes.c_double), ("drift_last", ctypes.c_double),
                ("numeric_err", ctypes.c_int32), ("learn_proposals", ctypes.c_int64),
                ("learn_accepted", ctypes.c_int64), ("phase_re", ctypes.c_double), ("phase_im", ctypes.c_double),
                ("phase_drift", ctypes.c_double)]


TIMING_CLASSES = ("wrap", "window", "expand", "flush", "stab", "measure", "learn")
FLUSH_KERNELS = ("direct", "tiled", "queue")
NET_NPARAM = 31170


class Timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * len(TIMING_CLASSES)), ("ms", ctypes.c_double * len(TIMING_CLASSES)),
                ("flush_flops", ctypes.c_double), ("wrap_bytes", ctypes.c_double)]


_P = ctypes.c_void_p
_SIGS = {
    "dqmc_workspace_size": [ctypes.POINTER(InstanceDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "dqmc_create": [ctypes.POINTER(InstanceDesc), ctypes.c_int32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "dqmc_destroy": [_P],
    "dqmc_set_fields": [_P, ctypes.c_int32, _P],
    "dqmc_get_fields": [_P, ctypes.c_int32, _P],
    "dqmc_sweep": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_replay": [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_get_green": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_set_green": [_P, ctypes.c_int32, _P],
    "dqmc_wrap": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_flush_test": [_P, ctypes.c_int32, _P, _P, ctypes.c_int32],
    "dqmc_measure": [_P, ctypes.c_int32, ctypes.POINTER(Obs)],
    "dqmc_reset_obs": [_P],
    "dqmc_set_measure_k": [_P, ctypes.c_int32],
    "dqmc_set_y_solver": [_P, ctypes.c_int32],
    "dqmc_set_expand_kernel": [_P, ctypes.c_int32],
    "dqmc_set_update_scheme": [_P, ctypes.c_int32],
    "dqmc_get_nk": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_get_series": [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "dqmc_measure_tau": [_P, ctypes.c_int32, _P],
    "dqmc_get_tau": [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_int64)],
    "dqmc_get_tau_rows": [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "dqmc_get_green_tau": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_tau_integrals": [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "dqmc_get_stats": [_P, ctypes.c_int32, ctypes.POINTER(Stats)],
    "dqmc_set_drift_tol": [_P, ctypes.c_double],
    "dqmc_shape": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                   ctypes.POINTER(ctypes.c_int32)],
    "dqmc_set_timing": [_P, ctypes.c_int32],
    "dqmc_get_timing": [_P, ctypes.POINTER(Timing)],
    "dqmc_set_proposals": [_P, ctypes.c_int32, ctypes.c_int32],
    "dqmc_net_set_weights": [_P, _P, ctypes.c_int64],
    "dqmc_net_get_weights": [_P, _P, ctypes.c_int64],
    "dqmc_net_init": [_P, ctypes.c_uint64],
    "dqmc_get_targets": [_P, ctypes.c_int32, _P],
    "dqmc_net_workspace_size": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_size_t)],
    "dqmc_net_logits": [_P, _P, ctypes.c_size_t, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_net_logits_noalloc": [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "dqmc_net_grad": [_P, _P, ctypes.c_size_t, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                      ctypes.c_int32, _P, _P],
    "dqmc_collect": [_P, ctypes.c_int32],
    "dqmc_sample_count": [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "dqmc_get_samples": [_P, ctypes.c_int64, ctypes.c_int32, _P, _P],
    "dqmc_net_train_workspace_size": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "dqmc_net_train": [_P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                       _P],
    "dqmc_set_delay": [_P, ctypes.c_int32],
    "dqmc_set_streams": [_P, ctypes.c_int32],
    "dqmc_set_graphs": [_P, ctypes.c_int32],
    "dqmc_autotune": [_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P],
    "dqmc_set_flush_kernel": [_P, ctypes.c_int32],
    "dqmc_set_fft_tile": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "dqmc_fft_plan_count": [_P, ctypes.POINTER(ctypes.c_int32), _P],
    "dqmc_autotune_fft": [_P, ctypes.c_int32, _P, _P],
    "dqmc_status_string": [ctypes.c_int32],
    "dqmc_last_error": [_P],
}

_lib = None


def load():
    """Load libdqmc.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdqmc.so is not built (run: python -m paper_2609_14668_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("dqmc_status_string", "dqmc_last_error") else ctypes.c_int32
    _lib = lib
    return lib


def _descs(descs):
    arr = (InstanceDesc * len(descs))()
    for i, d in enumerate(descs):
        for k, _ in InstanceDesc._fields_:
            setattr(arr[i], k, d.get(k, 0) if k == "channel" else d[k])
    return arr


def dqmc_workspace_size(descs):
    lib = load()
    arr = _descs(descs)
    out = ctypes.c_size_t(0)
    st = lib.dqmc_workspace_size(arr, len(descs), ctypes.byref(out))
    if st != DQMC_OK:
        raise DqmcError(st, "workspace_size")
    return out.value


def dqmc_tau_integrals(c, dtau, n_sites, degree=-1):
    """(dD/dU, chi_F) from C_{H_I}(l dtau), l = 0 .. n-1 (last point beta/2):
    degree < 0 trapezoid rule, else the integrated least-squares polynomial."""
    lib = load()
    buf = np.ascontiguousarray(c, dtype=np.float64)
    d, x = ctypes.c_double(), ctypes.c_double()
    st = lib.dqmc_tau_integrals(buf.ctypes.data, len(buf), float(dtau), int(n_sites), int(degree),
                                ctypes.byref(d), ctypes.byref(x))
    if st != DQMC_OK:
        raise DqmcError(st, "tau_integrals")
    return d.value, x.value


tau_integrals = dqmc_tau_integrals


class Simulation:
    """A handle over a batch of Markov chains (one dict per chain, keys as in
    dqmc_instance_desc).  The workspace is a torch uint8 tensor on the GPU."""

    def __init__(self, descs, device="cuda"):
        import torch
        self.lib = load()
        self.descs = [dict(d) for d in descs]
        self._arr = _descs(self.descs)
        size = dqmc_workspace_size(self.descs)
        self.ws = torch.empty(size + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(self.ws.device)
        h = _P()
        st = self.lib.dqmc_create(self._arr, len(descs), self._ws_ptr, size, self.stream.cuda_stream,
                                  ctypes.byref(h))
        if st != DQMC_OK:
            raise DqmcError(st, "dqmc_create")
        self.h = h
        self.n = len(descs)
        self.shapes = [self.shape(i) for i in range(self.n)]

    # ---- helpers
    def _chk(self, st, what):
        if st != DQMC_OK:
            msg = self.lib.dqmc_last_error(self.h)
            raise DqmcError(st, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        if getattr(self, "h", None):
            self.lib.dqmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, inst):
        N = ctypes.c_int32()
        M = ctypes.c_int32()
        c = ctypes.c_int32()
        self._chk(self.lib.dqmc_shape(self.h, inst, ctypes.byref(N), ctypes.byref(M), ctypes.byref(c)), "shape")
        return N.value, M.value, bool(c.value)

    # ---- C entry points
    def dqmc_sweep(self, n_sweeps, measure=True):
        self._chk(self.lib.dqmc_sweep(self.h, n_sweeps, int(bool(measure)), None), "sweep")

    sweep = dqmc_sweep

    def dqmc_replay(self, bits, ratios=None, n_sweeps=1, measure=False):
        """bits: torch.uint8 CUDA tensor [n_inst, bits_per_inst]; ratios: float64 same shape or None."""
        bits = bits.contiguous()
        rp = ratios.data_ptr() if ratios is not None else None
        self._chk(self.lib.dqmc_replay(self.h, bits.data_ptr(), bits.shape[1], rp, n_sweeps, int(bool(measure)),
                                       None), "replay")

    replay = dqmc_replay

    def dqmc_get_green(self, inst=0, spin=0):
        N, _, cx = self.shapes[inst]
        out = np.empty((N, N, 2) if cx else (N, N), dtype=np.float64)
        self._chk(self.lib.dqmc_get_green(self.h, inst, spin, out.ctypes.data), "get_green")
        return out[..., 0] + 1j * out[..., 1] if cx else out

    green = dqmc_get_green

    def dqmc_set_green(self, inst, G):
        N, _, cx = self.shapes[inst]
        if cx:
            buf = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1), dtype=np.float64)
        else:
            buf = np.ascontiguousarray(np.real(G), dtype=np.float64)
        self._chk(self.lib.dqmc_set_green(self.h, inst, buf.ctypes.data), "set_green")

    set_green = dqmc_set_green

    def dqmc_get_fields(self, inst=0):
        N, M, _ = self.shapes[inst]
        out = np.empty((M, N), dtype=np.int8)
        self._chk(self.lib.dqmc_get_fields(self.h, inst, out.ctypes.data), "get_fields")
        return out

    fields = dqmc_get_fields

    def dqmc_set_fields(self, inst, x):
        x = np.ascontiguousarray(x, dtype=np.int8)
        self._chk(self.lib.dqmc_set_fields(self.h, inst, x.ctypes.data), "set_fields")

    set_fields = dqmc_set_fields

    def dqmc_wrap(self, direction, slice_):
        self._chk(self.lib.dqmc_wrap(self.h, direction, slice_, None), "wrap")

    wrap = dqmc_wrap

    def dqmc_flush_test(self, inst, X, Y):
        N, _, cx = self.shapes[inst]
        k = X.shape[1]

        def pack(A):
            if cx:
                return np.ascontiguousarray(np.stack([A.real, A.imag], axis=-1), dtype=np.float64)
            return np.ascontiguousarray(np.real(A), dtype=np.float64)
        Xb = pack(np.asfortranarray(X).T.copy())      # column j contiguous (column-major N x k)
        Yb = pack(np.ascontiguousarray(Y))            # row m contiguous (k x N)
        self._chk(self.lib.dqmc_flush_test(self.h, inst, Xb.ctypes.data, Yb.ctypes.data, k), "flush_test")

    flush_test = dqmc_flush_test

    def dqmc_measure(self, inst=0):
        o = Obs()
        self._chk(self.lib.dqmc_measure(self.h, inst, ctypes.byref(o)), "measure")
        d = {f: getattr(o, f) for f in OBS_FIELDS}
        d["n_meas"] = o.n_meas
        return d

    measure = dqmc_measure

    def dqmc_set_update_scheme(self, scheme):
        """0: delayed update (default); 1: submatrix update (one block update per window)."""
        self._chk(self.lib.dqmc_set_update_scheme(self.h, int(scheme)), "set_update_scheme")

    set_update_scheme = dqmc_set_update_scheme

    def dqmc_set_expand_kernel(self, mm):
        """0: window vectors by the recursion (default); 1: in matrix form."""
        self._chk(self.lib.dqmc_set_expand_kernel(self.h, int(mm)), "set_expand_kernel")

    set_expand_kernel = dqmc_set_expand_kernel

    def dqmc_set_y_solver(self, lu):
        """1: Y^{-1} by pivoted LU (default); 0: by Householder QR."""
        self._chk(self.lib.dqmc_set_y_solver(self.h, int(lu)), "set_y_solver")

    set_y_solver = dqmc_set_y_solver

    def dqmc_set_measure_k(self, on):
        self._chk(self.lib.dqmc_set_measure_k(self.h, int(bool(on))), "set_measure_k")

    set_measure_k = dqmc_set_measure_k

    def dqmc_get_nk(self, inst=0, raw=False):
        """raw: complex (N_c, 2, 2) mean n(k); else a dict of the columns
        eps (|f|), n_AA, n_BB, n_AB (complex), n_plus, n_minus."""
        Nc = self.shapes[inst][0] // 2
        out = np.zeros(Nc * (8 if raw else 7), dtype=np.float64)
        self._chk(self.lib.dqmc_get_nk(self.h, inst, int(bool(raw)), out.ctypes.data), "get_nk")
        if raw:
            m = out.reshape(Nc, 2, 2, 2)
            return m[..., 0] + 1j * m[..., 1]
        m = out.reshape(Nc, 7)
        return {"eps": m[:, 0], "n_AA": m[:, 1], "n_BB": m[:, 2], "n_AB": m[:, 3] + 1j * m[:, 4],
                "n_plus": m[:, 5], "n_minus": m[:, 6]}

    nk = dqmc_get_nk

    def dqmc_reset_obs(self):
        self._chk(self.lib.dqmc_reset_obs(self.h), "reset_obs")

    reset_obs = dqmc_reset_obs

    def dqmc_get_series(self, inst=0, max_sweeps=4096):
        out = np.zeros((max_sweeps, len(SERIES_FIELDS)), dtype=np.float64)
        n = ctypes.c_int32()
        self._chk(self.lib.dqmc_get_series(self.h, inst, out.ctypes.data, max_sweeps, ctypes.byref(n)), "series")
        return {f: out[:n.value, k].copy() for k, f in enumerate(SERIES_FIELDS)}

    series = dqmc_get_series

    def dqmc_measure_tau(self, l_max=-1):
        self._chk(self.lib.dqmc_measure_tau(self.h, int(l_max), None), "measure_tau")

    measure_tau = dqmc_measure_tau

    def dqmc_get_tau(self, inst=0):
        """(<A(tau_l) A(0)>, <A> at slice l, for l = 0..M/2; number of passes)."""
        M = self.shapes[inst][1]
        aa = np.zeros(M // 2 + 1, dtype=np.float64)
        at = np.zeros(M // 2 + 1, dtype=np.float64)
        n = ctypes.c_int64()
        self._chk(self.lib.dqmc_get_tau(self.h, inst, aa.ctypes.data, at.ctypes.data, ctypes.byref(n)), "get_tau")
        return aa, at, n.value

    get_tau = dqmc_get_tau

    def dqmc_get_tau_rows(self, inst=0, max_rows=1024):
        """Per pass: columns 0..M/2 <A(tau_l) A(0)>_X, then M/2+1.. <A>_X(tau_l)."""
        M = self.shapes[inst][1]
        out = np.zeros((max_rows, 2 * (M // 2) + 2), dtype=np.float64)
        n = ctypes.c_int32()
        self._chk(self.lib.dqmc_get_tau_rows(self.h, inst, out.ctypes.data, max_rows, ctypes.byref(n)), "tau_rows")
        return out[:n.value].copy()

    tau_rows = dqmc_get_tau_rows

    def dqmc_get_green_tau(self, inst=0, which=1):
        N, _, cx = self.shapes[inst]
        out = np.empty((N, N, 2) if cx else (N, N), dtype=np.float64)
        self._chk(self.lib.dqmc_get_green_tau(self.h, inst, which, out.ctypes.data), "get_green_tau")
        return out[..., 0] + 1j * out[..., 1] if cx else out

    green_tau = dqmc_get_green_tau

    def dqmc_get_stats(self, inst=0, check=False):
        """Counters of one instance.  DQMC_ENUMERIC still fills them: it is
        raised only with check=True, else reported in numeric_err."""
        s = Stats()
        st = self.lib.dqmc_get_stats(self.h, inst, ctypes.byref(s))
        if st != DQMC_OK and (check or st != -4):
            self._chk(st, "stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    stats = dqmc_get_stats

    def dqmc_set_drift_tol(self, tol):
        self._chk(self.lib.dqmc_set_drift_tol(self.h, float(tol)), "set_drift_tol")

    set_drift_tol = dqmc_set_drift_tol

    def dqmc_set_timing(self, on=True):
        self._chk(self.lib.dqmc_set_timing(self.h, int(bool(on))), "set_timing")

    set_timing = dqmc_set_timing

    def dqmc_get_timing(self):
        t = Timing()
        self._chk(self.lib.dqmc_get_timing(self.h, ctypes.byref(t)), "get_timing")
        out = {c: {"launches": t.launches[i], "ms": t.ms[i]} for i, c in enumerate(TIMING_CLASSES)}
        out["flush_flops"] = t.flush_flops
        out["wrap_bytes"] = t.wrap_bytes
        return out

    timing = dqmc_get_timing

    # ---- learned multi-site moves and the proposal network
    def dqmc_set_proposals(self, per_slice, m):
        self._chk(self.lib.dqmc_set_proposals(self.h, int(per_slice), int(m)), "set_proposals")

    set_proposals = dqmc_set_proposals

    def dqmc_net_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._chk(self.lib.dqmc_net_set_weights(self.h, w.ctypes.data, w.size), "net_set_weights")

    net_set_weights = dqmc_net_set_weights

    def dqmc_net_init(self, seed=1):
        self._chk(self.lib.dqmc_net_init(self.h, int(seed)), "net_init")

    net_init = dqmc_net_init

    def dqmc_net_get_weights(self):
        w = np.empty(NET_NPARAM, dtype=np.float32)
        self._chk(self.lib.dqmc_net_get_weights(self.h, w.ctypes.data, w.size), "net_get_weights")
        return w

    net_get_weights = dqmc_net_get_weights

    def dqmc_get_targets(self, inst=0):
        N, M, _ = self.shapes[inst]
        out = np.empty((M, N), dtype=np.float32)
        self._chk(self.lib.dqmc_get_targets(self.h, inst, out.ctypes.data), "get_targets")
        return out

    targets = dqmc_get_targets

    def _net_ws(self, L, M, n_samples, batch):
        import torch
        size = ctypes.c_size_t(0)
        self._chk(self.lib.dqmc_net_workspace_size(L, M, n_samples, batch, ctypes.byref(size)), "net_workspace_size")
        key = (size.value,)
        if getattr(self, "_nws_key", None) != key:
            self._nws = torch.empty(size.value + 256, dtype=torch.uint8, device=self.ws.device)
            self._nws_key = key
        ptr = (self._nws.data_ptr() + 255) & ~255
        return ptr, size.value

    def dqmc_net_logits(self, fields, L):
        """fields: int8 (n, M, N) -> logits float32 (n, M, N)."""
        x = np.ascontiguousarray(fields, dtype=np.int8)
        n, M, N = x.shape
        ptr, size = self._net_ws(L, M, n, n)
        out = np.empty((n, M, N), dtype=np.float32)
        self._chk(self.lib.dqmc_net_logits(self.h, ptr, size, x.ctypes.data, n, L, M, out.ctypes.data), "net_logits")
        return out

    net_logits = dqmc_net_logits

    def dqmc_net_logits_noalloc(self, fields, L):
        """As net_logits, with the library's static device scratch (no
        device allocation in the call)."""
        x = np.ascontiguousarray(fields, dtype=np.int8)
        n, M, N = x.shape
        out = np.empty((n, M, N), dtype=np.float32)
        self._chk(self.lib.dqmc_net_logits_noalloc(self.h, x.ctypes.data, n, L, M, out.ctypes.data),
                  "net_logits_noalloc")
        return out

    net_logits_noalloc = dqmc_net_logits_noalloc

    def dqmc_net_grad(self, fields, targets, L, window=False):
        """window=False: configurations (n, M, N) with targets (n, M, N);
        window=True: 7-slice windows (n, 7, N) with centre targets (n, N)."""
        x = np.ascontiguousarray(fields, dtype=np.int8)
        t = np.ascontiguousarray(targets, dtype=np.float32)
        n, M, N = x.shape
        ptr, size = self._net_ws(L, M, n, n)
        loss = ctypes.c_float(0)
        g = np.empty(NET_NPARAM, dtype=np.float32)
        self._chk(self.lib.dqmc_net_grad(self.h, ptr, size, x.ctypes.data, t.ctypes.data, n, L, M, int(bool(window)),
                                         ctypes.byref(loss), g.ctypes.data), "net_grad")
        return loss.value, g

    net_grad = dqmc_net_grad

    def dqmc_collect(self, every):
        self._chk(self.lib.dqmc_collect(self.h, int(every)), "collect")

    collect = dqmc_collect

    def dqmc_sample_count(self):
        f = ctypes.c_int64()
        c = ctypes.c_int64()
        self._chk(self.lib.dqmc_sample_count(self.h, ctypes.byref(f), ctypes.byref(c)), "sample_count")
        return f.value, c.value

    sample_count = dqmc_sample_count

    def dqmc_get_samples(self, first, count):
        nmax = max(s[0] for s in self.shapes)
        win = np.empty((count, 7, nmax), dtype=np.int8)
        tg = np.empty((count, nmax), dtype=np.float32)
        self._chk(self.lib.dqmc_get_samples(self.h, int(first), int(count), win.ctypes.data, tg.ctypes.data),
                  "get_samples")
        return win, tg

    get_samples = dqmc_get_samples

    def dqmc_net_train(self, steps, batch=8, lr=1e-3, seed=1):
        import torch
        size = ctypes.c_size_t(0)
        self._chk(self.lib.dqmc_net_train_workspace_size(self.h, batch, ctypes.byref(size)), "net_train_ws")
        buf = torch.empty(size.value + 256, dtype=torch.uint8, device=self.ws.device)
        ptr = (buf.data_ptr() + 255) & ~255
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        self._chk(self.lib.dqmc_net_train(self.h, ptr, size.value, int(steps), int(batch), float(lr), int(seed),
                                          losses.ctypes.data), "net_train")
        return losses[:steps]

    net_train = dqmc_net_train

    def dqmc_set_delay(self, k):
        self._chk(self.lib.dqmc_set_delay(self.h, int(k)), "set_delay")

    set_delay = dqmc_set_delay

    def dqmc_autotune(self, candidates, steps):
        """Time `steps` slice steps per candidate flush rank and flush kernel
        and keep the fastest; returns ((k, kernel), {(k, kernel): ms per step})."""
        c = np.ascontiguousarray(candidates, dtype=np.int32)
        nv = len(FLUSH_KERNELS)
        ms = np.zeros(nv * c.size, dtype=np.float64)
        best = np.zeros(2, dtype=np.int32)
        self._chk(self.lib.dqmc_autotune(self.h, int(steps), c.ctypes.data, c.size, best.ctypes.data,
                                         ms.ctypes.data), "autotune")
        per = {(int(k), v): float(ms[nv * q + v]) for q, k in enumerate(c) for v in range(nv)
               if ms[nv * q + v] > 0}
        return (int(best[0]), int(best[1])), per

    def dqmc_set_flush_kernel(self, variant):
        self._chk(self.lib.dqmc_set_flush_kernel(self.h, int(variant)), "set_flush_kernel")

    set_flush_kernel = dqmc_set_flush_kernel

    autotune = dqmc_autotune

    def dqmc_set_fft_tile(self, L, side, tile):
        self._chk(self.lib.dqmc_set_fft_tile(self.h, int(L), int(side), int(tile)), "set_fft_tile")

    set_fft_tile = dqmc_set_fft_tile

    def dqmc_autotune_fft(self, reps=20):
        """Pick the register-line FFT tile per (L, side); returns
        ({(L, side): tile}, {(L, side, tile): microseconds})."""
        n = ctypes.c_int32(0)
        Ls = np.zeros(16, dtype=np.int32)
        self._chk(self.lib.dqmc_fft_plan_count(self.h, ctypes.byref(n), Ls.ctypes.data), "fft_plan_count")
        tiles = np.zeros(2 * max(n.value, 1), dtype=np.int32)
        us = np.zeros(6 * max(n.value, 1), dtype=np.float64)
        self._chk(self.lib.dqmc_autotune_fft(self.h, int(reps), tiles.ctypes.data, us.ctypes.data), "autotune_fft")
        choice = {(int(Ls[q]), side): int(tiles[2 * q + side]) for q in range(n.value) for side in (0, 1)}
        times = {(int(Ls[q]), side, t): float(us[(2 * q + side) * 3 + t])
                 for q in range(n.value) for side in (0, 1) for t in range(3)}
        return choice, times

    autotune_fft = dqmc_autotune_fft

    def dqmc_set_streams(self, groups):
        self._chk(self.lib.dqmc_set_streams(self.h, int(groups)), "set_streams")

    set_streams = dqmc_set_streams

    def dqmc_set_graphs(self, on):
        self._chk(self.lib.dqmc_set_graphs(self.h, int(bool(on))), "set_graphs")

    set_graphs = dqmc_set_graphs
