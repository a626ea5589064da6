"""ctypes binding of libpfft.so (see include/pfft.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (``data_ptr()``) and the HIP stream.
The library must be built (``python -m paper_2210_04891_amd.build``); there is
no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfft.so")

PFFT_FAR_ONLY = 1
PFFT_NEAR_ONLY = 2
PFFT_PRECOND = 4
PFFT_PRECOND_ONLY = 8
PFFT_LEARNED_ONLY = 16
MLP_MAGIC = 0x504D4C50

STATUS = {0: "PFFT_OK", -1: "PFFT_EINVAL", -2: "PFFT_ETOPO", -3: "PFFT_ENOMEM",
          -4: "PFFT_EDEVICE", -5: "PFFT_ENOCONV", -6: "PFFT_EFACTOR"}

EXPORTS = ("pfft_setup", "pfft_sizes", "pfft_matvec", "solve_ports", "extract_RL",
           "pfft_precond_load", "pfft_destroy", "pfft_last_error",
           "pfft_host_setup", "pfft_host_get", "pfft_host_free", "pfft_ctx_get", "pfft_profile",
           "pfft_stage_times", "pfft_precond_save", "pfft_learned_collect", "pfft_learned_train",
           "pfft_learned_clear", "pfft_learned_stats", "pfft_mlp_grad", "pfft_learned_eval",
           "pfft_set_option", "pfft_get_option", "pfft_autotune", "solve_ports_lgmres",
           "solve_ports_loops", "pfft_postprocess", "pfft_matvec_noalloc")

STAGES = ("loop_to_branch", "tri_current", "project", "fft_x", "fft_y", "fft_z_conv", "ifft_y",
          "ifft_x", "interp", "combine", "branch_to_loop", "precond")


class PfftError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("V", ctypes.c_void_p),
                ("nt", ctypes.c_int32), ("T", ctypes.c_void_p),
                ("nport", ctypes.c_int32),
                ("src_off", ctypes.c_void_p), ("src_tri", ctypes.c_void_p),
                ("snk_off", ctypes.c_void_p), ("snk_tri", ctypes.c_void_p),
                ("sigma", ctypes.c_double), ("mu_r", ctypes.c_double),
                ("grid", ctypes.c_int32 * 3), ("stencil", ctypes.c_int32),
                ("near_kappa", ctypes.c_double),
                ("grid_fp64", ctypes.c_int32), ("contact_zs", ctypes.c_int32),
                ("max_rhs_chunk", ctypes.c_int32)]


_lib = None


def load():
    """Load libpfft.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpfft.so is not built (run python -m paper_2210_04891_amd.build)")
    # PyTorch, which provides the callers' device memory and streams, is
    # loaded first: on a process whose first HIP call came from this library
    # without it, the runtime has reported no device
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.pfft_setup.argtypes = [ctypes.POINTER(_Problem), vp, ctypes.POINTER(vp)]
    lib.pfft_setup.restype = i32
    lib.pfft_sizes.argtypes = [vp, ctypes.POINTER(i64)]
    lib.pfft_sizes.restype = i32
    lib.pfft_matvec.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp]
    lib.pfft_matvec.restype = i32
    lib.pfft_matvec_noalloc.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp]
    lib.pfft_matvec_noalloc.restype = i32
    lib.solve_ports.argtypes = [vp, i32, vp, dbl, i32, i32, i32, vp, vp, vp, vp]
    lib.solve_ports.restype = i32
    lib.solve_ports_lgmres.argtypes = [vp, i32, vp, dbl, i32, i32, i32, vp, vp, vp, vp]
    lib.solve_ports_lgmres.restype = i32
    lib.solve_ports_loops.argtypes = [vp, i32, vp, dbl, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.solve_ports_loops.restype = i32
    lib.pfft_postprocess.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pfft_postprocess.restype = i32
    lib.extract_RL.argtypes = [i32, i32, vp, vp, vp, vp]
    lib.extract_RL.restype = i32
    lib.pfft_precond_load.argtypes = [vp, vp, i64]
    lib.pfft_precond_load.restype = i32
    lib.pfft_destroy.argtypes = [vp]
    lib.pfft_destroy.restype = None
    lib.pfft_last_error.argtypes = []
    lib.pfft_last_error.restype = ctypes.c_char_p
    lib.pfft_host_setup.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(vp)]
    lib.pfft_host_setup.restype = i32
    lib.pfft_host_get.argtypes = [vp, ctypes.c_char_p, vp, i64, ctypes.POINTER(i64)]
    lib.pfft_host_get.restype = i32
    lib.pfft_ctx_get.argtypes = [vp, ctypes.c_char_p, vp, i64, ctypes.POINTER(i64)]
    lib.pfft_ctx_get.restype = i32
    lib.pfft_host_free.argtypes = [vp]
    lib.pfft_host_free.restype = None
    lib.pfft_profile.argtypes = [vp, i32]
    lib.pfft_profile.restype = i32
    lib.pfft_stage_times.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.pfft_stage_times.restype = i32
    lib.pfft_precond_save.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    lib.pfft_precond_save.restype = i32
    lib.pfft_learned_collect.argtypes = [vp, i32, vp, dbl, i32, ctypes.POINTER(i64), vp]
    lib.pfft_learned_collect.restype = i32
    lib.pfft_learned_train.argtypes = [vp, i32, i32, i32, dbl, ctypes.c_uint64, vp, vp]
    lib.pfft_learned_train.restype = i32
    lib.pfft_set_option.argtypes = [vp, ctypes.c_char_p, i64]
    lib.pfft_set_option.restype = i32
    lib.pfft_get_option.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64)]
    lib.pfft_get_option.restype = i32
    lib.pfft_autotune.argtypes = [vp, i32, vp, i32, ctypes.c_char_p, i64, vp]
    lib.pfft_autotune.restype = i32
    lib.pfft_learned_eval.argtypes = [vp, ctypes.POINTER(dbl), vp]
    lib.pfft_learned_eval.restype = i32
    lib.pfft_learned_clear.argtypes = [vp]
    lib.pfft_learned_clear.restype = i32
    lib.pfft_learned_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.pfft_learned_stats.restype = i32
    lib.pfft_mlp_grad.argtypes = [i32, vp, i64, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    lib.pfft_mlp_grad.restype = i32
    _lib = lib
    return lib


def _check(code, allow=()):
    if code != 0 and code not in allow:
        raise PfftError(code, load().pfft_last_error().decode())
    return code


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _problem(structure, grid, stencil, near_kappa, grid_fp64, sigma, mu_r, contact_zs,
         max_rhs_chunk):
    V = np.ascontiguousarray(structure.V, dtype=np.float64)
    T = np.ascontiguousarray(structure.T, dtype=np.int32)
    ports = list(structure.ports)
    so = np.zeros(len(ports) + 1, np.int32)
    ko = np.zeros(len(ports) + 1, np.int32)
    for k, (s, t) in enumerate(ports):
        so[k + 1] = so[k] + len(s)
        ko[k + 1] = ko[k] + len(t)
    st = np.ascontiguousarray(np.concatenate([np.asarray(s, np.int32) for s, _ in ports])
                              if ports else np.zeros(1, np.int32), dtype=np.int32)
    kt = np.ascontiguousarray(np.concatenate([np.asarray(t, np.int32) for _, t in ports])
                              if ports else np.zeros(1, np.int32), dtype=np.int32)
    keep = (V, T, so, ko, st, kt)
    pb = _Problem()
    pb.nv, pb.V = V.shape[0], V.ctypes.data
    pb.nt, pb.T = T.shape[0], T.ctypes.data
    pb.nport = len(ports)
    pb.src_off, pb.src_tri = so.ctypes.data, st.ctypes.data
    pb.snk_off, pb.snk_tri = ko.ctypes.data, kt.ctypes.data
    pb.sigma, pb.mu_r = sigma, mu_r
    for d in range(3):
        pb.grid[d] = int(grid[d])
    pb.stencil = stencil
    pb.near_kappa = near_kappa
    pb.grid_fp64 = 1 if grid_fp64 else 0
    pb.contact_zs = 1 if contact_zs else 0
    pb.max_rhs_chunk = max_rhs_chunk
    return pb, keep


class HostModel:
    """Host-only setup (pfft_host_setup): topology, loop basis, Gram, grid
    weights and near-field CSR, for inspection without a GPU."""

    def __init__(self, structure, grid, stencil=4, near_kappa=1.5, contact_zs=False):
        lib = load()
        pb, self._keep = _problem(structure, grid, stencil, near_kappa, False, 5.8e7, 1.0,
                                  contact_zs, 0)
        h = ctypes.c_void_p()
        _check(lib.pfft_host_setup(ctypes.byref(pb), ctypes.byref(h)))
        self._h = h

    def get(self, name, dtype):
        lib = load()
        n = ctypes.c_int64()
        _check(lib.pfft_host_get(self._h, name.encode(), None, 0, ctypes.byref(n)))
        out = np.empty(n.value // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib.pfft_host_get(self._h, name.encode(), ctypes.c_void_p(out.ctypes.data),
                                 n.value, ctypes.byref(n)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().pfft_host_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A set-up problem (pfft_setup).  ``structure`` needs V (nv x 3, metres),
    T (n x 3) and ports [(src_tris, snk_tris), ...]."""

    def __init__(self, structure, grid, stencil=4, near_kappa=1.5, grid_fp64=False,
                 sigma=5.8e7, mu_r=1.0, contact_zs=False, max_rhs_chunk=0, stream=None):
        lib = load()
        pb, self._keep = _problem(structure, grid, stencil, near_kappa, grid_fp64, sigma, mu_r,
                                  contact_zs, max_rhs_chunk)
        ports = list(structure.ports)
        h = ctypes.c_void_p()
        _check(lib.pfft_setup(ctypes.byref(pb), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.nport = len(ports)
        self.sizes = self._sizes()

    def _sizes(self):
        out = (ctypes.c_int64 * 10)()
        _check(load().pfft_sizes(self._h, out))
        keys = ("n", "nprime", "b", "l", "s", "p", "nnz_near", "Ng", "near_pairs", "device_bytes")
        return dict(zip(keys, [int(v) for v in out]))

    def matvec(self, x, omega=None, space=1, flags=0, out=None, stream=None):
        """y = op(x); x is a complex128 CUDA tensor [R, dim]."""
        import torch
        assert x.dtype == torch.complex128 and x.is_cuda and x.dim() == 2
        x = x.contiguous()
        R = x.shape[0]
        dim = self.sizes["l"] if space == 1 else self.sizes["b"]
        if x.shape[1] != dim:
            raise ValueError("x has %d columns, expected %d" % (x.shape[1], dim))
        y = torch.empty_like(x) if out is None else out
        om = None
        if space == 1:
            om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, np.float64), (R,)))
        _check(load().pfft_matvec(self._h, R, _ptr(om) if om is not None else None, space, flags,
                                  ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  _stream_handle(stream)))
        return y

    def matvec_noalloc(self, x, omega=None, space=1, flags=0, out=None, stream=None):
        """matvec through pfft_matvec_noalloc (no device allocation inside
        the call; the library's fixed scratch holds the workspace); y must be
        given or is allocated here, before the call."""
        import torch
        assert x.dtype == torch.complex128 and x.is_cuda and x.dim() == 2
        x = x.contiguous()
        R = x.shape[0]
        dim = self.sizes["l"] if space == 1 else self.sizes["b"]
        if x.shape[1] != dim:
            raise ValueError("x has %d columns, expected %d" % (x.shape[1], dim))
        y = torch.empty_like(x) if out is None else out
        om = None
        if space == 1:
            om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, np.float64), (R,)))
        _check(load().pfft_matvec_noalloc(self._h, R, _ptr(om) if om is not None else None, space, flags,
                                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                          _stream_handle(stream)))
        return y

    def solve_ports(self, freqs_hz, tol=1e-6, maxit=500, restart=60, precond=1, stream=None):
        """Right-preconditioned FGMRES.  Returns (Y [nf, p, p] complex128,
        iterations [nf, p], relres [nf, p], status)."""
        return self._solve(load().solve_ports, freqs_hz, tol, maxit, restart, precond, stream)

    def solve_ports_lgmres(self, freqs_hz, tol=1e-3, maxit=500, restart=60, precond=1, stream=None):
        """Left-preconditioned GMRES (relres is the preconditioned residual).
        Returns as solve_ports."""
        return self._solve(load().solve_ports_lgmres, freqs_hz, tol, maxit, restart, precond, stream)

    def solve_ports_loops(self, freqs_hz, tol=1e-6, maxit=500, restart=60, precond=1, stream=None):
        """solve_ports that also returns the loop currents, a device complex128
        tensor [nf * p, l] (row f * p + k: port k driven at frequency f).
        Returns (Y, iterations, relres, status, I_l)."""
        import torch
        f = np.ascontiguousarray(np.asarray(freqs_hz, np.float64).reshape(-1))
        Il = torch.empty((f.size * self.nport, self.sizes["l"]), dtype=torch.complex128, device="cuda")
        lib = load()

        def fn(h, nf, fp, tol_, maxit_, restart_, pre, Yp, itp, rrp, st):
            return lib.solve_ports_loops(h, nf, fp, tol_, maxit_, restart_, pre, Yp, itp, rrp,
                                         ctypes.c_void_p(Il.data_ptr()), st)
        Y, it, rr, code = self._solve(fn, f, tol, maxit, restart, precond, stream)
        return Y, it, rr, code, Il

    def postprocess(self, Il, omega, stream=None):
        """Sec. V-A outputs of loop currents Il (device complex128 [R, l]) at
        omega [R] (rad/s): dict of device tensors Vl [R, l], Ib [R, b + p],
        Vb [R, b], J [R, n, 3], phi [R, n]."""
        import torch
        assert Il.dtype == torch.complex128 and Il.is_cuda and Il.dim() == 2
        if Il.shape[1] != self.sizes["l"]:
            raise ValueError("Il has %d columns, expected %d" % (Il.shape[1], self.sizes["l"]))
        Il = Il.contiguous()
        R = Il.shape[0]
        om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(-1))
        if om.size != R:
            raise ValueError("omega must have one value per row of Il")
        n, b, l, p = self.sizes["n"], self.sizes["b"], self.sizes["l"], self.nport
        kw = dict(dtype=torch.complex128, device=Il.device)
        out = dict(Vl=torch.empty((R, l), **kw), Ib=torch.empty((R, b + p), **kw), Vb=torch.empty((R, b), **kw),
                   J=torch.empty((R, n, 3), **kw), phi=torch.empty((R, n), **kw))
        vp_ = ctypes.c_void_p
        _check(load().pfft_postprocess(self._h, R, _ptr(om), vp_(Il.data_ptr()), vp_(out["Vl"].data_ptr()),
                                       vp_(out["Ib"].data_ptr()), vp_(out["Vb"].data_ptr()),
                                       vp_(out["J"].data_ptr()), vp_(out["phi"].data_ptr()),
                                       _stream_handle(stream)))
        return out

    def _solve(self, fn, freqs_hz, tol, maxit, restart, precond, stream):
        f = np.ascontiguousarray(np.asarray(freqs_hz, np.float64).reshape(-1))
        nf, p = f.size, self.nport
        Y = np.zeros((nf, p, p), np.complex128)
        it = np.zeros((nf, p), np.int32)
        rr = np.zeros((nf, p), np.float64)
        code = _check(fn(self._h, nf, _ptr(f), tol, maxit, restart, precond,
                         _ptr(Y), _ptr(it), _ptr(rr), _stream_handle(stream)),
                      allow=(-5,))
        return Y, it, rr, code

    def set_option(self, name, value):
        """Plan options: fft_plan, ldl_plan, project_plan, graphs (0 or 1)."""
        _check(load().pfft_set_option(self._h, name.encode(), int(value)))

    def model_array(self, name, dtype):
        """A named array of the context's host model (pfft_ctx_get)."""
        lib = load()
        n = ctypes.c_int64()
        _check(lib.pfft_ctx_get(self._h, name.encode(), None, 0, ctypes.byref(n)))
        out = np.empty(n.value // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib.pfft_ctx_get(self._h, name.encode(), ctypes.c_void_p(out.ctypes.data), n.value,
                                ctypes.byref(n)))
        return out

    def get_option(self, name):
        v = ctypes.c_int64()
        _check(load().pfft_get_option(self._h, name.encode(), ctypes.byref(v)))
        return v.value

    def autotune(self, omega, reps=3, stream=None):
        """Time each plan on the preconditioned product for len(omega)
        right-hand sides, keep the fastest; returns the report (dict)."""
        import json
        om = np.ascontiguousarray(np.asarray(omega, np.float64).reshape(-1))
        buf = ctypes.create_string_buffer(4096)
        _check(load().pfft_autotune(self._h, om.size, _ptr(om), reps, buf, len(buf), _stream_handle(stream)))
        return json.loads(buf.value.decode())

    def profile(self, enable=True):
        _check(load().pfft_profile(self._h, 1 if enable else 0))

    def stage_times(self):
        """{stage: (total ms, launches)} since the last profile() call."""
        ms = (ctypes.c_double * 16)()
        calls = (ctypes.c_int64 * 16)()
        _check(load().pfft_stage_times(self._h, ms, calls))
        return {name: (ms[i], int(calls[i])) for i, name in enumerate(STAGES)}

    def precond_load(self, blob):
        """Load a weight blob (bytes or uint8 array, layout in pfft.h)."""
        w = np.frombuffer(bytes(blob), np.uint8).copy()
        _check(load().pfft_precond_load(self._h, _ptr(w), w.nbytes))

    def precond_save(self):
        """Current weight blob as bytes."""
        n = ctypes.c_int64()
        _check(load().pfft_precond_save(self._h, None, 0, ctypes.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        _check(load().pfft_precond_save(self._h, _ptr(buf), n.value, ctypes.byref(n)))
        return buf.tobytes()

    def learned_collect(self, freqs_hz, tol=1e-8, maxit=60, stream=None):
        """Append (Krylov vector, exact error) training pairs from one-cycle
        plain-P solves; returns the training-set size in rows."""
        f = np.ascontiguousarray(np.asarray(freqs_hz, np.float64).reshape(-1))
        rows = ctypes.c_int64()
        _check(load().pfft_learned_collect(self._h, f.size, _ptr(f), tol, maxit,
                                           ctypes.byref(rows), _stream_handle(stream)))
        return rows.value

    def learned_train(self, steps, batch=8192, hidden=256, lr=1e-3, seed=0, stream=None):
        """Adam steps on the collected set; returns the per-step minibatch loss."""
        loss = np.zeros(max(steps, 1), np.float32)
        _check(load().pfft_learned_train(self._h, steps, batch, hidden, lr, seed, _ptr(loss),
                                         _stream_handle(stream)))
        return loss[:steps]

    def learned_eval(self, stream=None):
        """Loss of the current network over the whole training set."""
        v = ctypes.c_double()
        _check(load().pfft_learned_eval(self._h, ctypes.byref(v), _stream_handle(stream)))
        return v.value

    def learned_clear(self):
        _check(load().pfft_learned_clear(self._h))

    def learned_stats(self):
        """(applications, numeric fallbacks to P^-1, right-hand sides switched
        back to plain P by the convergence judge)."""
        out = (ctypes.c_int64 * 3)()
        _check(load().pfft_learned_stats(self._h, out))
        return int(out[0]), int(out[1]), int(out[2])

    def close(self):
        if getattr(self, "_h", None):
            load().pfft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _to_bf16_bits(a):
    """float -> bfloat16 bit patterns (round to nearest even)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def mlp_blob(params):
    """Weight blob (pfft.h layout) from {W1 [H,F], W2 [H,H], W3 [O,H], b1, b2, b3}."""
    W1, W2, W3 = (np.asarray(params[k], np.float64) for k in ("W1", "W2", "W3"))
    H, F = W1.shape
    O = W3.shape[0]
    w = _to_bf16_bits(np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()]))
    if w.size % 2:
        w = np.concatenate([w, np.zeros(1, np.uint16)])
    b = np.concatenate([np.asarray(params[k], np.float32).ravel() for k in ("b1", "b2", "b3")])
    head = np.array([MLP_MAGIC, F, H, O], np.uint32).view(np.int32)
    return head.tobytes() + w.tobytes() + b.astype(np.float32).tobytes()


def mlp_params(blob):
    """Inverse of mlp_blob (weights as the float64 values of their bf16)."""
    raw = bytes(blob)
    magic, F, H, O = np.frombuffer(raw[:16], np.int32)
    if np.uint32(magic) != MLP_MAGIC:
        raise ValueError("not a weight blob")
    nw = H * F + H * H + O * H
    w = np.frombuffer(raw[16:16 + 2 * nw], np.uint16).astype(np.uint32) << 16
    w = w.view(np.float32).astype(np.float64)
    off = 16 + 4 * ((nw + 1) // 2)
    b = np.frombuffer(raw[off:], np.float32).astype(np.float64)
    return dict(W1=w[:H * F].reshape(H, F), W2=w[H * F:H * F + H * H].reshape(H, H),
                W3=w[H * F + H * H:].reshape(O, H), b1=b[:H], b2=b[H:2 * H], b3=b[2 * H:])


def mlp_grad(blob, X_bf16, T, w, stream=None):
    """Network output, loss sum_i w_i |y_i - t_i|^2 and parameter gradients
    on the device (pfft_mlp_grad).  X_bf16: CUDA int16/uint16 tensor [rows, F]
    of bf16 bit patterns (or torch.bfloat16); T: float32 [rows, 2]; w: float32
    [rows].  Returns (Y [rows, 2] float32 tensor, gradient dict, loss)."""
    import torch
    raw = np.frombuffer(bytes(blob), np.uint8).copy()
    _, F, H, O = np.frombuffer(raw[:16].tobytes(), np.int32)
    rows = X_bf16.shape[0]
    Y = torch.empty((rows, 2), dtype=torch.float32, device=X_bf16.device)
    npar = H * F + H * H + 2 * H + 2 * H + 2
    g = torch.empty(npar, dtype=torch.float32, device=X_bf16.device)
    loss = ctypes.c_double()
    X_bf16, T, w = X_bf16.contiguous(), T.contiguous(), w.contiguous()
    _check(load().pfft_mlp_grad(rows, _ptr(raw), raw.nbytes, ctypes.c_void_p(X_bf16.data_ptr()),
                                ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                ctypes.byref(loss), _stream_handle(stream)))
    gc = g.cpu().numpy().astype(np.float64)
    sizes = [("W1", (H, F)), ("W2", (H, H)), ("W3", (2, H)), ("b1", (H,)), ("b2", (H,)), ("b3", (2,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = gc[o:o + n].reshape(shp)
        o += n
    return Y, out, loss.value


def extract_RL(freqs_hz, Y):
    f = np.ascontiguousarray(np.asarray(freqs_hz, np.float64).reshape(-1))
    Y = np.ascontiguousarray(Y, dtype=np.complex128)
    nf, p = Y.shape[0], Y.shape[1]
    R = np.zeros((nf, p, p))
    L = np.zeros((nf, p, p))
    _check(load().extract_RL(nf, p, _ptr(f), _ptr(Y), _ptr(R), _ptr(L)))
    return R, L
