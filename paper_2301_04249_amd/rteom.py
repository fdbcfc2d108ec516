"""ctypes binding of the C ABI declared in include/rteom.h.

Argument marshalling only: every step of the hot path runs in the HIP library
``librteom.so`` built in this directory.  PyTorch is used for the device
workspace and the stream; importing this module never falls back to any other
implementation -- if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librteom.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_HIP", 4: "ERR_NOCONV", 5: "ERR_NONFINITE",
          6: "ERR_STATE"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}

# every exported symbol of include/rteom.h
SYMBOLS = (
    "rteom_default_options", "rteom_workspace_query", "rteom_init", "rteom_step", "rteom_cumulant",
    "rteom_spectral", "rteom_spectral_noalloc", "rteom_spectral_peaks", "rteom_ground_state", "rteom_checkpoint", "rteom_restore", "rteom_dims", "rteom_set_amplitudes", "rteom_get_amplitudes", "rteom_residual", "rteom_energy",
    "rteom_residual_flops", "rteom_plan_info", "rteom_device_sets", "rteom_profile", "rteom_phase_stats",
    "rteom_tile_cache_save", "rteom_tile_cache_load", "rteom_batch_create",
    "rteom_batch_step",
    "rteom_batch_free", "rteom_free", "rteom_last_error",
)
PHASES = ("ladder", "ring", "gemm", "move", "update", "energy", "build")


class RteomError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("prec", ctypes.c_int32),
        ("fp_map", ctypes.c_int32),
        ("fp_fixed_iters", ctypes.c_int32),
        ("fp_max_iter", ctypes.c_int32),
        ("fp_tol", ctypes.c_double),
        ("dC_include_fT1", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("max_steps", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("tune", ctypes.c_int32),
        ("fp_anderson", ctypes.c_int32),
        ("mem_limit", ctypes.c_size_t),
        ("plan_slab", ctypes.c_int32),
        ("plan_block", ctypes.c_int32),
        ("progress", ctypes.c_int32),
    ]


_LIBS = {}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def load(path: str = LIB_PATH):
    """Load (once) the library at ``path`` and declare the ABI signatures."""
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise RuntimeError(f"RT-EOM-CCSD library not built: {path} is missing (run __graft_entry__.build())")
    # One HIP runtime per process: torch bundles its own libamdhip64.so.7.  Loading
    # torch first makes the library's libamdhip64.so.7 dependency resolve to that
    # already-loaded runtime, so device memory and streams are shared with torch.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - host-only use (workspace queries)
        pass
    lib = ctypes.CDLL(path)
    c = ctypes
    lib.rteom_default_options.argtypes = [c.POINTER(Options)]
    lib.rteom_default_options.restype = None
    lib.rteom_workspace_query.argtypes = [c.c_int32] * 6 + [c.POINTER(Options), c.POINTER(c.c_size_t)]
    lib.rteom_init.argtypes = [c.POINTER(c.c_void_p), c.c_int32, c.c_int32, c.c_int32, _dp, c.c_int32, _dp,
                               c.c_int32, c.c_int32, c.POINTER(Options)]
    lib.rteom_step.argtypes = [c.c_void_p, c.c_double, c.c_int32, _ip]
    lib.rteom_cumulant.argtypes = [c.c_void_p, c.c_int64, _dp, _dp, c.POINTER(c.c_int64)]
    lib.rteom_spectral.argtypes = [c.c_void_p, c.c_double, c.c_double, c.c_int64, _dp, _dp, _dp]
    lib.rteom_spectral_noalloc.argtypes = [c.c_void_p, c.c_double, c.c_double, c.c_int64, _dp, _dp, _dp]
    lib.rteom_spectral_peaks.argtypes = [c.c_void_p, c.c_double, c.c_double, c.c_int64, _dp, _dp, c.c_int32, _dp,
                                         _ip]
    lib.rteom_ground_state.argtypes = [c.c_void_p, c.c_double, c.c_int32, _dp, _ip]
    lib.rteom_checkpoint.argtypes = [c.c_void_p, c.c_void_p, c.c_size_t, c.POINTER(c.c_size_t)]
    lib.rteom_restore.argtypes = [c.c_void_p, c.c_void_p, c.c_size_t]
    lib.rteom_dims.argtypes = [c.c_void_p, _ip, _ip, _ip, _ip]
    lib.rteom_set_amplitudes.argtypes = [c.c_void_p, _dp, _dp]
    lib.rteom_get_amplitudes.argtypes = [c.c_void_p, _dp, _dp]
    lib.rteom_residual.argtypes = [c.c_void_p, _dp, _dp]
    lib.rteom_energy.argtypes = [c.c_void_p, _dp]
    lib.rteom_residual_flops.argtypes = [c.c_void_p, _dp]
    lib.rteom_device_sets.argtypes = [c.c_void_p, c.POINTER(c.c_void_p), c.POINTER(c.c_void_p),
                                      c.POINTER(c.c_int64)]
    lib.rteom_plan_info.argtypes = [c.c_void_p, _ip, c.POINTER(c.c_int64), c.POINTER(c.c_int64),
                                    c.POINTER(c.c_int64), _dp, c.POINTER(c.c_size_t)]
    lib.rteom_profile.argtypes = [c.c_void_p, c.c_uint32]
    lib.rteom_phase_stats.argtypes = [c.c_void_p, c.c_int32, _dp, _dp, c.POINTER(c.c_int64)]
    lib.rteom_tile_cache_save.argtypes = [c.c_void_p, c.c_char_p]
    lib.rteom_tile_cache_load.argtypes = [c.c_void_p, c.c_char_p]
    lib.rteom_batch_create.argtypes = [c.POINTER(c.c_void_p), c.c_int32, c.POINTER(c.c_void_p)]
    lib.rteom_batch_step.argtypes = [c.c_void_p, c.c_double, c.c_int32]
    lib.rteom_batch_free.argtypes = [c.c_void_p]
    lib.rteom_free.argtypes = [c.c_void_p]
    lib.rteom_last_error.argtypes = [c.c_void_p]
    lib.rteom_last_error.restype = c.c_char_p
    for name in SYMBOLS:
        if name not in ("rteom_default_options", "rteom_last_error"):
            getattr(lib, name).restype = c.c_int
    _LIBS[path] = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def pair_index(n):
    """(first, second) index arrays of the pairs i < j of n in the ABI's lexicographic order."""
    i, j = np.triu_indices(n, 1)
    return i, j


def pack_same_spin(full):
    """[n1][n1][n2][n2] antisymmetric block -> its pair storage [P1][P2] (elements i < j, a < b)."""
    n1, n2 = full.shape[0], full.shape[2]
    i, j = pair_index(n1)
    a, b = pair_index(n2)
    return np.ascontiguousarray(full[i, j][:, a, b])


def expand_same_spin(pairs, n1, n2):
    """Pair storage [P1][P2] -> the full antisymmetric block [n1][n1][n2][n2] (layout only:
    each stored element and its sign-flipped images)."""
    out = np.zeros((n1, n1, n2, n2), dtype=pairs.dtype)
    i, j = pair_index(n1)
    a, b = pair_index(n2)
    blk = np.zeros((len(i), n2, n2), dtype=pairs.dtype)
    blk[:, a, b] = pairs
    blk[:, b, a] = -pairs
    out[i, j] = blk
    out[j, i] = -blk
    return out


class Propagator:
    """One core-hole propagation (rteom_init ... rteom_free)."""

    def __init__(self, eps, chol, n_occ_a, n_occ_b, core_orb=0, core_spin=1, prec="fp64", fp_map=0,
                 fixed_iters=0, max_iter=50, tol=1e-10, include_ft1=True, max_steps=100000,
                 stream=None, workspace=None, graph=False, tune=True, anderson=0, mem_limit=0, plan_slab=0, plan_block=0, progress=False,
                 lib_path=LIB_PATH):
        self.lib = load(lib_path)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        chol = np.ascontiguousarray(chol, dtype=np.float64)
        nq, n, n2 = chol.shape
        assert n == n2 == eps.shape[0]
        opt = Options()
        self.lib.rteom_default_options(ctypes.byref(opt))
        opt.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        opt.fp_map = int(fp_map)
        opt.fp_fixed_iters = int(fixed_iters)
        opt.fp_max_iter = int(max_iter)
        opt.fp_tol = float(tol)
        opt.dC_include_fT1 = 1 if include_ft1 else 0
        opt.max_steps = int(max_steps)
        opt.graph = 1 if graph else 0
        opt.tune = 1 if tune else 0
        opt.fp_anderson = int(anderson)
        opt.mem_limit = int(mem_limit)
        opt.plan_slab = int(plan_slab)
        opt.plan_block = int(plan_block)
        opt.progress = 1 if progress else 0
        opt.stream = stream
        self._ws = None
        if workspace in ("torch", "torch-cpu"):
            # "torch-cpu": host memory, for the library's host test build only
            import torch
            need = ctypes.c_size_t(0)
            st = self.lib.rteom_workspace_query(n, n_occ_a, n_occ_b, nq, core_orb, core_spin, ctypes.byref(opt),
                                                ctypes.byref(need))
            self._check(st, None)
            self._ws = torch.empty(int(need.value), dtype=torch.uint8,
                                   device="cuda" if workspace == "torch" else "cpu")
            opt.workspace = self._ws.data_ptr()
            opt.workspace_bytes = int(need.value)
            if stream is None and workspace == "torch":
                if graph:   # a stream of its own (at the default priority) so that it can be captured
                    self._stream = torch.cuda.Stream()
                    opt.stream = self._stream.cuda_stream
                else:
                    opt.stream = torch.cuda.current_stream().cuda_stream
        self.opt = opt
        h = ctypes.c_void_p()
        st = self.lib.rteom_init(ctypes.byref(h), n, n_occ_a, n_occ_b, _ptr(eps), nq, _ptr(chol), core_orb,
                                 core_spin, ctypes.byref(opt))
        self._check(st, None)
        self.h = h
        no, nv = ctypes.c_int32(), ctypes.c_int32()
        self.lib.rteom_dims(self.h, ctypes.byref(no), ctypes.byref(nv), None, None)
        self.no, self.nv = no.value, nv.value
        occ = np.zeros(self.no, dtype=np.int32)
        vir = np.zeros(self.nv, dtype=np.int32)
        self.lib.rteom_dims(self.h, None, None, occ.ctypes.data_as(_ip), vir.ctypes.data_as(_ip))
        self.occ_list, self.vir_list = occ, vir

    def _check(self, st, h):
        if st != 0:
            msg = self.lib.rteom_last_error(h)
            raise RteomError(st, msg.decode() if msg else "")

    # -- amplitude layout helpers (host; include/rteom.h): t1 [2][n_o][n_v], t2 = the two
    # same-spin blocks in pair storage [2][P_o][P_v] followed by the alpha-beta block
    # [n_o][n_o][n_v][n_v].  Methods take and return t2 either as that pair (tss, tab) or,
    # with full=True, as the antisymmetric full blocks [3][n_o][n_o][n_v][n_v] (aa, ab, bb).
    def t1_shape(self):
        return (2, self.no, self.nv)

    def t2_shape(self):
        return (3, self.no, self.no, self.nv, self.nv)

    def _t2_flat(self, t2):
        no, nv = self.no, self.nv
        if isinstance(t2, tuple):
            tss, tab = t2
        else:
            t2 = np.asarray(t2)
            tss = np.stack([pack_same_spin(t2[0]), pack_same_spin(t2[2])])
            tab = t2[1]
        po, pv = no * (no - 1) // 2, nv * (nv - 1) // 2
        tss = np.asarray(tss, dtype=np.complex128).reshape(2 * po * pv)
        tab = np.asarray(tab, dtype=np.complex128).reshape(no * no * nv * nv)
        return np.ascontiguousarray(np.concatenate([tss, tab]))

    def _t2_out(self, flat, full):
        no, nv = self.no, self.nv
        po, pv = no * (no - 1) // 2, nv * (nv - 1) // 2
        tss = flat[: 2 * po * pv].reshape(2, po, pv)
        tab = flat[2 * po * pv:].reshape(no, no, nv, nv)
        if not full:
            return tss, tab
        return np.stack([expand_same_spin(tss[0], no, nv), tab, expand_same_spin(tss[1], no, nv)])

    def device_sets(self):
        """(x, r): float64 torch views of the device amplitude set and residual set inside the
        torch workspace (rteom_device_sets; workspace="torch" only), planar device layout."""
        x, r, n = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        st = self.lib.rteom_device_sets(self.h, ctypes.byref(x), ctypes.byref(r), ctypes.byref(n))
        self._check(st, self.h)
        if self._ws is None:
            raise RteomError(1, "device_sets needs workspace='torch'")
        base = self._ws.data_ptr()
        views = []
        for p in (x.value, r.value):
            off = p - base
            views.append(self._ws[off: off + 8 * n.value].view(__import__("torch").float64))
        return views[0], views[1]

    def amplitudes_written(self):
        """The device amplitude set was written in place: mask it and recompute E(T_n)."""
        st = self.lib.rteom_set_amplitudes(self.h, None, None)
        self._check(st, self.h)

    def plan(self):
        """The memory plan rteom_init chose (rteom_plan_info)."""
        res, es, cj, ci = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        fl, ws = ctypes.c_double(), ctypes.c_size_t()
        st = self.lib.rteom_plan_info(self.h, ctypes.byref(res), ctypes.byref(es), ctypes.byref(cj), ctypes.byref(ci),
                                      ctypes.byref(fl), ctypes.byref(ws))
        self._check(st, self.h)
        return {"resident": bool(res.value), "e_slab": es.value, "ring_cols": cj.value, "rows": ci.value,
                "exec_flops": fl.value, "workspace_bytes": ws.value}

    def step(self, dt, n_steps=1):
        iters = np.zeros(max(n_steps, 1), dtype=np.int32)
        st = self.lib.rteom_step(self.h, float(dt), int(n_steps), iters.ctypes.data_as(_ip))
        self._check(st, self.h)
        return iters[:n_steps]

    def cumulant(self):
        """(times, C) for t_0 = 0 ... t_n (rteom_cumulant)."""
        n = ctypes.c_int64()
        st = self.lib.rteom_cumulant(self.h, 0, None, None, ctypes.byref(n))   # query the length
        self._check(st, self.h)
        total = n.value
        t = np.zeros(max(total, 1))
        c = np.zeros((max(total, 1), 2))
        st = self.lib.rteom_cumulant(self.h, total, _ptr(t), _ptr(c), ctypes.byref(n))
        self._check(st, self.h)
        return t[: n.value], c[: n.value, 0] + 1j * c[: n.value, 1]

    def ground_state(self, tol=1e-10, max_iter=200):
        """(E^corr, iterations) of ground-state CCSD for this reference (rteom_ground_state);
        create the propagator with core_orb=-1 for the N-electron determinant."""
        e = np.zeros(2)
        it = ctypes.c_int32()
        st = self.lib.rteom_ground_state(self.h, float(tol), int(max_iter), _ptr(e), ctypes.byref(it))
        self._check(st, self.h)
        return complex(e[0], e[1]), it.value

    def checkpoint(self):
        """Image of the propagation state (amplitudes, C/E histories, times) as bytes."""
        n = ctypes.c_size_t()
        st = self.lib.rteom_checkpoint(self.h, None, 0, ctypes.byref(n))
        self._check(st, self.h)
        buf = ctypes.create_string_buffer(n.value)
        st = self.lib.rteom_checkpoint(self.h, buf, n.value, ctypes.byref(n))
        self._check(st, self.h)
        return buf.raw

    def restore(self, image):
        """Continue from an image written by checkpoint() (same system)."""
        data = bytes(image)
        st = self.lib.rteom_restore(self.h, data, len(data))
        self._check(st, self.h)

    def spectral(self, omegas, eta, e_corr=0.0, noalloc=False):
        """(A(omega), qp position, A at the grid maximum) from the device C(t) (rteom_spectral, or
        rteom_spectral_noalloc with noalloc=True)."""
        w = np.ascontiguousarray(omegas, dtype=np.float64)
        a = np.zeros(w.shape[0])
        qp = np.zeros(2)
        fn = self.lib.rteom_spectral_noalloc if noalloc else self.lib.rteom_spectral
        st = fn(self.h, float(e_corr), float(eta), w.shape[0], _ptr(w), _ptr(a), _ptr(qp))
        self._check(st, self.h)
        return a, qp[0], qp[1]

    def _n2(self):
        no, nv = self.no, self.nv
        return no * (no - 1) * nv * (nv - 1) // 2 + no * no * nv * nv

    def spectral_peaks(self, omegas, eta, max_peaks=8, e_corr=0.0):
        """(A(omega), peaks [n][2] = (position, height), largest first) (rteom_spectral_peaks)."""
        w = np.ascontiguousarray(omegas, dtype=np.float64)
        a = np.zeros(w.shape[0])
        pk = np.zeros((max_peaks, 2))
        n = ctypes.c_int32()
        st = self.lib.rteom_spectral_peaks(self.h, float(e_corr), float(eta), w.shape[0], _ptr(w), _ptr(a),
                                           int(max_peaks), _ptr(pk), ctypes.byref(n))
        self._check(st, self.h)
        return a, pk[: n.value].copy()

    def set_amplitudes(self, t1, t2):
        t1 = np.ascontiguousarray(t1, dtype=np.complex128).reshape(self.t1_shape())
        t2 = self._t2_flat(t2)
        st = self.lib.rteom_set_amplitudes(self.h, t1.view(np.float64).ctypes.data_as(_dp),
                                           t2.view(np.float64).ctypes.data_as(_dp))
        self._check(st, self.h)

    def get_amplitudes(self, full=True):
        t1 = np.zeros(self.t1_shape(), dtype=np.complex128)
        t2 = np.zeros(self._n2(), dtype=np.complex128)
        st = self.lib.rteom_get_amplitudes(self.h, t1.view(np.float64).ctypes.data_as(_dp),
                                           t2.view(np.float64).ctypes.data_as(_dp))
        self._check(st, self.h)
        return t1, self._t2_out(t2, full)

    def residual(self, want=True, full=True):
        if not want:
            st = self.lib.rteom_residual(self.h, None, None)
            self._check(st, self.h)
            return None
        r1 = np.zeros(self.t1_shape(), dtype=np.complex128)
        r2 = np.zeros(self._n2(), dtype=np.complex128)
        st = self.lib.rteom_residual(self.h, r1.view(np.float64).ctypes.data_as(_dp),
                                     r2.view(np.float64).ctypes.data_as(_dp))
        self._check(st, self.h)
        return r1, self._t2_out(r2, full)

    def energy(self):
        e = np.zeros(2)
        st = self.lib.rteom_energy(self.h, _ptr(e))
        self._check(st, self.h)
        return complex(e[0], e[1])

    def residual_flops(self):
        f = ctypes.c_double()
        st = self.lib.rteom_residual_flops(self.h, ctypes.byref(f))
        self._check(st, self.h)
        return f.value

    def profile(self, phases=()):
        """Time the named phases (see PHASES) with HIP events on the library's stream."""
        mask = 0
        for ph in phases:
            mask |= 1 << PHASES.index(ph)
        st = self.lib.rteom_profile(self.h, mask)
        self._check(st, self.h)

    def phase_stats(self, phase):
        """(device ms since the last query, ops timed, flops of this phase per residual)."""
        ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        st = self.lib.rteom_phase_stats(self.h, PHASES.index(phase), ctypes.byref(ms), ctypes.byref(fl),
                                        ctypes.byref(n))
        self._check(st, self.h)
        return ms.value, n.value, fl.value

    def save_tiles(self, path):
        """Write the context's timed tile choices to a file (rteom_tile_cache_save)."""
        self._check(self.lib.rteom_tile_cache_save(self.h, os.fsencode(path)), self.h)

    def load_tiles(self, path):
        """Add a file's tile choices to the context (rteom_tile_cache_load)."""
        self._check(self.lib.rteom_tile_cache_load(self.h, os.fsencode(path)), self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rteom_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several propagations advanced together, each one's captured step replayed on its own stream (rteom_batch_*)."""

    def __init__(self, props):
        self.props = list(props)
        self.lib = self.props[0].lib
        arr = (ctypes.c_void_p * len(self.props))(*[p.h.value for p in self.props])
        h = ctypes.c_void_p()
        st = self.lib.rteom_batch_create(ctypes.byref(h), len(self.props), arr)
        if st != 0:
            raise RteomError(st, self.lib.rteom_last_error(None).decode())
        self.h = h

    def step(self, dt, n_steps=1):
        st = self.lib.rteom_batch_step(self.h, float(dt), int(n_steps))
        if st != 0:
            raise RteomError(st, self.lib.rteom_last_error(None).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rteom_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
