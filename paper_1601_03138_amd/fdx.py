"""ctypes binding of libfdx.so (include/fdx.h): argument marshalling only.

Every step of the force path runs in the HIP library; this module never computes forces,
keys or lists itself and has no CPU fallback: if the library is missing it raises.
PyTorch is used only for device memory (tensors passed by pointer) and streams.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdx.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4
MEM_HOST, MEM_DEVICE = 0, 1
QUAD, FP32REL, PREDICTOR, PERSISTENT, GRAPH, TIMING, FUSED = 1, 2, 4, 8, 16, 32, 64
CUT_FIXED, CUT_SCATTER, CUT_GATHER, CUT_SYMMETRIC = 0, 1, 2, 3
DD_COST_LISTS = 1

EXPORTS = ["fdx_create", "fdx_destroy", "fdx_set_particles", "fdx_build_tree", "fdx_calc_force",
           "fdx_integrate", "fdx_get_particles", "fdx_get_forces", "fdx_get_stats",
           "fdx_get_tree", "fdx_get_groups", "fdx_get_lists", "fdx_last_error",
           "fdx_autotune_shapes", "fdx_shape_name", "fdx_set_shape", "fdx_autotune", "fdx_mlp_params",
           "fdx_predictor_features", "fdx_mlp_forward", "fdx_mlp_grad", "fdx_mlp_adam",
           "fdx_predictor_train",
           "fdx_predictor_margin", "fdx_predictor_save", "fdx_predictor_load",
           "fdx_build_exchange_lists", "fdx_get_exchange_counts", "fdx_get_exchange_lists",
           "fdx_get_exchange_stats", "fdx_calc_density", "fdx_get_density",
           "fdx_calc_force_cutoff", "fdx_dd_factor", "fdx_decompose", "fdx_get_decomposition",
           "fdx_get_dd_samples", "fdx_get_dd_destinations", "fdx_exchange_particles",
           "fdx_get_dd_stats", "fdx_direct_forces", "fdx_autotune_cached",
           "fdx_set_graph_list_margin", "fdx_calc_force_noalloc", "fdx_set_list_capture"]


class FdxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdx error {code}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n", "n_sys", "n_cells", "n_groups", "depth", "n_epj", "n_spj", "n_interactions_pp",
        "n_interactions_pc", "overflow_groups", "list_capacity")] + [
        ("n_leaf", C.c_int32), ("n_group", C.c_int32), ("flags", C.c_int32),
        ("shape", C.c_int32), ("theta", C.c_double)] + [(k, C.c_double) for k in (
            "t_keys", "t_sort", "t_tree", "t_moments", "t_groups", "t_walk", "t_force",
            "t_unsort", "t_predict", "t_total")] + [("fp64_groups", C.c_int64),
                                                    ("graph_recoveries", C.c_int64),
                                                    ("list_spills", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ExchangeStats(C.Structure):
    _fields_ = [("n_domains", C.c_int64), ("n_pairs", C.c_int64), ("n_epj", C.c_int64),
                ("n_spj", C.c_int64), ("list_capacity", C.c_int64), ("ms_tree", C.c_double),
                ("ms_lists", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class DdStats(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("n_domains", C.c_int32), ("n_src", C.c_int32), ("n_samples", C.c_int64),
                ("n_moved", C.c_int64), ("ms_sample", C.c_double), ("ms_divide", C.c_double),
                ("ms_assign", C.c_double), ("ms_exchange", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def load() -> C.CDLL:
    """Load the built library (raises if it has not been built: there is no fallback)."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime with the same soname; loading it first makes this
        # library bind to that one runtime, so torch's streams and allocations are shared.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise FdxError(ESTATE, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        _declare(lib)
        _LIB = lib
    return _LIB


def _declare(L):
    vp, i64, i32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.fdx_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.fdx_destroy.argtypes = [vp]
    L.fdx_set_particles.argtypes = [vp, i64] + [vp] * 9 + [i32, i32]
    L.fdx_build_tree.argtypes = [vp, i32, i32]
    L.fdx_calc_force.argtypes = [vp, f64, i32, i32, f64, i32]
    L.fdx_integrate.argtypes = [vp, f64, i32, i32]
    L.fdx_get_particles.argtypes = [vp] + [vp] * 6 + [i32]
    L.fdx_get_forces.argtypes = [vp] + [vp] * 4 + [i32]
    L.fdx_get_stats.argtypes = [vp, C.POINTER(Stats)]
    L.fdx_get_tree.argtypes = [vp] + [vp] * 11
    L.fdx_get_groups.argtypes = [vp] + [vp] * 6
    L.fdx_get_lists.argtypes = [vp] + [vp] * 4
    L.fdx_last_error.argtypes = [vp]
    L.fdx_last_error.restype = C.c_char_p
    L.fdx_autotune_shapes.argtypes = []
    L.fdx_set_shape.argtypes = [vp, i32]
    L.fdx_set_graph_list_margin.argtypes = [vp, i32]
    L.fdx_set_list_capture.argtypes = [vp, i32]
    L.fdx_shape_name.argtypes = [i32]
    L.fdx_shape_name.restype = C.c_char_p
    L.fdx_autotune.argtypes = [vp, f64, i32, f64, i32, vp, i32, i32, vp, vp, vp]
    L.fdx_mlp_params.argtypes = []
    L.fdx_predictor_features.argtypes = [vp, vp]
    L.fdx_mlp_forward.argtypes = [vp, vp, vp, i64, vp]
    L.fdx_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    L.fdx_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i32, i32, f64]
    L.fdx_predictor_train.argtypes = [vp, vp, vp, i64, i32, i32, f64, i64, vp]
    L.fdx_predictor_margin.argtypes = [vp, f64, vp]
    L.fdx_predictor_save.argtypes = [vp, C.c_char_p]
    L.fdx_predictor_load.argtypes = [vp, C.c_char_p]
    L.fdx_build_exchange_lists.argtypes = [vp, f64, i32]
    L.fdx_get_exchange_counts.argtypes = [vp, vp, vp]
    L.fdx_get_exchange_lists.argtypes = [vp, vp, vp]
    L.fdx_get_exchange_stats.argtypes = [vp, C.POINTER(ExchangeStats)]
    L.fdx_calc_density.argtypes = [vp, i32, f64, vp, i32, i32, i32, i32]
    L.fdx_calc_force_cutoff.argtypes = [vp, f64, i32, i32, f64, f64, i32]
    L.fdx_get_density.argtypes = [vp, vp, vp, i32]
    L.fdx_dd_factor.argtypes = [i32, vp, vp, vp]
    L.fdx_decompose.argtypes = [vp, i32, i32, i32, i64, vp, C.c_uint64, i32]
    L.fdx_get_decomposition.argtypes = [vp] + [vp] * 5
    L.fdx_get_dd_samples.argtypes = [vp] + [vp] * 3
    L.fdx_get_dd_destinations.argtypes = [vp, vp, vp, i32]
    L.fdx_exchange_particles.argtypes = [vp]
    L.fdx_get_dd_stats.argtypes = [vp, C.POINTER(DdStats)]
    L.fdx_direct_forces.argtypes = [vp, vp, i64, f64, vp]
    L.fdx_autotune_cached.argtypes = [vp, C.c_char_p, f64, i32, f64, i32, vp, i32, i32, vp, vp,
                                      vp]
    L.fdx_calc_force_noalloc.argtypes = [C.c_int, vp, i64] + [vp] * 5 + [f64, f64, i32, i32, i32] \
        + [vp] * 4 + [C.c_char_p, i32]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Context:
    """One library context bound to a device and a HIP stream (torch's current stream by
    default when torch is importable and a GPU is present, else a library-owned stream)."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        handle = C.c_void_p()
        s = None
        if stream is not None:
            s = C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        rc = self.lib.fdx_create(C.byref(handle), device, s)
        if rc != OK:
            raise FdxError(rc, f"fdx_create(device={device}) failed")
        self.h = handle
        self.n = 0
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.fdx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int, what: str):
        if rc != OK:
            msg = self.lib.fdx_last_error(self.h)
            raise FdxError(rc, f"{what}: {msg.decode() if msg else ''}")

    # -- particles -------------------------------------------------------------------
    def set_particles(self, ps, per_particle_eps: bool = True):
        """Copy a ParticleSet (numpy FP64 arrays) to the device."""
        arrs = [_f64(getattr(ps, k)) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]
        eps = _f64(ps.eps) if per_particle_eps else None
        off = None if ps.sys_off is None else np.ascontiguousarray(ps.sys_off, dtype=np.int64)
        n_sys = 1 if off is None else off.shape[0] - 1
        self._check(self.lib.fdx_set_particles(self.h, ps.n, *[_ptr(a) for a in arrs], _ptr(eps),
                                               _ptr(off), n_sys, MEM_HOST), "set_particles")
        self.n = ps.n
        self._keep = []

    def set_particles_device(self, tensors: dict, sys_off=None):
        """Borrow device tensors (torch FP64, contiguous): keys x, y, z, vx, vy, vz, m, eps
        (eps optional).  The tensors must stay alive while the context uses them."""
        ts = [tensors[k] for k in ("x", "y", "z", "vx", "vy", "vz", "m")]
        n = int(ts[0].numel())
        for t in ts:
            if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64"
                    and t.numel() == n):
                raise ValueError("device tensors must be contiguous float64 CUDA tensors of one length")
        eps = tensors.get("eps")
        off = None if sys_off is None else np.ascontiguousarray(sys_off, dtype=np.int64)
        n_sys = 1 if off is None else off.shape[0] - 1
        self._check(self.lib.fdx_set_particles(self.h, n, *[_dptr(t) for t in ts], _dptr(eps),
                                               _ptr(off), n_sys, MEM_DEVICE), "set_particles")
        self.n = n
        self._keep = list(ts) + ([eps] if eps is not None else [])

    # -- evaluation ------------------------------------------------------------------
    @staticmethod
    def flags(quad=True, fp32=False, predictor=False, persistent=False, timing=False,
              fused=False) -> int:
        return ((QUAD if quad else 0) | (FP32REL if fp32 else 0) | (PREDICTOR if predictor else 0)
                | (PERSISTENT if persistent else 0) | (TIMING if timing else 0)
                | (FUSED if fused else 0))

    def set_list_capture(self, on: bool):
        """FDX_FUSED evaluations also store the lists they evaluate (for checks)."""
        self._check(self.lib.fdx_set_list_capture(self.h, 1 if on else 0), "set_list_capture")

    def build_tree(self, n_leaf: int = 8, n_group: int = 64):
        self._check(self.lib.fdx_build_tree(self.h, n_leaf, n_group), "build_tree")

    def calc_force(self, theta: float = 0.5, n_leaf: int = 8, n_group: int = 64,
                   eps: float = 0.0, **kw):
        self._check(self.lib.fdx_calc_force(self.h, float(theta), n_leaf, n_group, float(eps),
                                            self.flags(**kw)), "calc_force")

    def calc_force_flags(self, theta, n_leaf, n_group, eps, flags: int):
        self._check(self.lib.fdx_calc_force(self.h, float(theta), n_leaf, n_group, float(eps),
                                            int(flags)), "calc_force")

    def integrate(self, dt: float, n_steps: int, graph: bool = False):
        self._check(self.lib.fdx_integrate(self.h, float(dt), int(n_steps), GRAPH if graph else 0),
                    "integrate")

    # -- results ---------------------------------------------------------------------
    def forces(self) -> np.ndarray:
        out = [np.empty(self.n) for _ in range(4)]
        self._check(self.lib.fdx_get_forces(self.h, *[_ptr(a) for a in out], MEM_HOST), "get_forces")
        return np.stack(out, axis=1)

    def forces_device(self, ax, ay, az, pot):
        self._check(self.lib.fdx_get_forces(self.h, _dptr(ax), _dptr(ay), _dptr(az), _dptr(pot),
                                            MEM_DEVICE), "get_forces")

    def particles(self):
        out = [np.empty(self.n) for _ in range(6)]
        self._check(self.lib.fdx_get_particles(self.h, *[_ptr(a) for a in out], MEM_HOST),
                    "get_particles")
        return out

    def stats(self) -> dict:
        st = Stats()
        self._check(self.lib.fdx_get_stats(self.h, C.byref(st)), "get_stats")
        return st.as_dict()

    def tree(self) -> dict:
        st = self.stats()
        nc, n, S = int(st["n_cells"]), self.n, int(st["n_sys"])
        d = dict(cube=np.empty((S, 4)), key=np.empty(n, np.uint64), perm=np.empty(n, np.uint32),
                 level=np.empty(nc, np.int32), prefix=np.empty(nc, np.uint64),
                 begin=np.empty(nc, np.uint32), count=np.empty(nc, np.uint32),
                 first_child=np.empty(nc, np.uint32), nchild=np.empty(nc, np.uint32),
                 parent=np.empty(nc, np.uint32), mom=np.empty((nc, 10)))
        order = ["cube", "key", "perm", "level", "prefix", "begin", "count", "first_child",
                 "nchild", "parent", "mom"]
        self._check(self.lib.fdx_get_tree(self.h, *[_ptr(d[k]) for k in order]), "get_tree")
        return d

    def groups(self) -> dict:
        G = int(self.stats()["n_groups"])
        d = dict(cell=np.empty(G, np.uint32), begin=np.empty(G, np.uint32),
                 count=np.empty(G, np.uint32), qmin=np.empty((G, 3), np.uint32),
                 qmax=np.empty((G, 3), np.uint32), centre=np.empty((G, 3)))
        order = ["cell", "begin", "count", "qmin", "qmax", "centre"]
        self._check(self.lib.fdx_get_groups(self.h, *[_ptr(d[k]) for k in order]), "get_groups")
        return d

    def list_counts(self):
        G = int(self.stats()["n_groups"])
        ne, ns = np.empty(G, np.uint32), np.empty(G, np.uint32)
        self._check(self.lib.fdx_get_lists(self.h, _ptr(ne), _ptr(ns), None, None), "get_lists")
        return ne, ns

    def lists(self):
        st = self.stats()
        G = int(st["n_groups"])
        ne, ns = np.empty(G, np.uint32), np.empty(G, np.uint32)
        epj = np.empty(max(1, int(st["n_epj"])), np.uint32)
        spj = np.empty(max(1, int(st["n_spj"])), np.uint32)
        self._check(self.lib.fdx_get_lists(self.h, _ptr(ne), _ptr(ns), _ptr(epj), _ptr(spj)),
                    "get_lists")
        return ne, ns, epj[:int(st["n_epj"])], spj[:int(st["n_spj"])]

    # -- autotuner ---------------------------------------------------------------------
    def autotune(self, theta, n_leaf, eps, flags, n_group_candidates, reps=2):
        cand = np.ascontiguousarray(n_group_candidates, dtype=np.int32)
        nv = self.lib.fdx_autotune_shapes()
        times = np.full(cand.shape[0] * nv, np.nan)
        bg, bv = C.c_int32(), C.c_int32()
        self._check(self.lib.fdx_autotune(self.h, float(theta), n_leaf, float(eps), int(flags),
                                          _ptr(cand), cand.shape[0], reps, _ptr(times),
                                          C.byref(bg), C.byref(bv)), "autotune")
        return int(bg.value), int(bv.value), times.reshape(cand.shape[0], nv)

    def autotune_cached(self, path, theta, n_leaf, eps, flags, n_group_candidates, reps=2):
        """(n_group, shape, from_cache): fdx_autotune with its result recorded in `path`."""
        cand = np.ascontiguousarray(n_group_candidates, dtype=np.int32)
        bg, bv, fc = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.fdx_autotune_cached(self.h, os.fsencode(str(path)), float(theta),
                                                 n_leaf, float(eps), int(flags), _ptr(cand),
                                                 cand.shape[0], reps, C.byref(bg), C.byref(bv),
                                                 C.byref(fc)), "autotune_cached")
        return int(bg.value), int(bv.value), bool(fc.value)

    def shape_name(self, shape: int) -> str:
        return self.lib.fdx_shape_name(int(shape)).decode()

    def set_shape(self, shape: int):
        self._check(self.lib.fdx_set_shape(self.h, int(shape)), "set_shape")

    def set_graph_list_margin(self, percent: int):
        """List segments of graph-captured steps with several systems: percent of each
        system's longest list (0: count walk every step)."""
        self._check(self.lib.fdx_set_graph_list_margin(self.h, int(percent)),
                    "set_graph_list_margin")

    # -- exchange lists between domains (the systems of the particle set) ----------------
    def build_exchange_lists(self, theta: float, n_leaf: int = 8):
        self._check(self.lib.fdx_build_exchange_lists(self.h, float(theta), int(n_leaf)),
                    "build_exchange_lists")

    def exchange_counts(self):
        """(n_epj, n_spj) as n_sys x n_sys matrices, row = sender, column = receiver."""
        S = int(self.stats()["n_sys"])
        ne, ns = np.empty(S * S, np.uint32), np.empty(S * S, np.uint32)
        self._check(self.lib.fdx_get_exchange_counts(self.h, _ptr(ne), _ptr(ns)),
                    "get_exchange_counts")
        return ne.reshape(S, S), ns.reshape(S, S)

    def exchange_lists(self):
        """(pairs, n_epj, n_spj, epj, spj): pairs in order (sender, receiver != sender),
        per-pair counts, and the concatenated entries (caller's particle indices, cell ids)."""
        ne, ns = self.exchange_counts()
        S = ne.shape[0]
        pairs = [(a, b) for a in range(S) for b in range(S) if b != a]
        pe = np.array([ne[a, b] for a, b in pairs], np.int64)
        psj = np.array([ns[a, b] for a, b in pairs], np.int64)
        epj = np.empty(max(1, int(pe.sum())), np.uint32)
        spj = np.empty(max(1, int(psj.sum())), np.uint32)
        self._check(self.lib.fdx_get_exchange_lists(self.h, _ptr(epj), _ptr(spj)),
                    "get_exchange_lists")
        return pairs, pe, psj, epj[:int(pe.sum())], spj[:int(psj.sum())]

    def exchange_stats(self) -> dict:
        st = ExchangeStats()
        self._check(self.lib.fdx_get_exchange_stats(self.h, C.byref(st)), "get_exchange_stats")
        return st.as_dict()

    # -- FP64 direct summation (reference) ------------------------------------------------
    def direct_forces(self, targets, eps: float = 0.0) -> np.ndarray:
        """[len(targets), 4] = (ax, ay, az, phi) by FP64 direct summation over each target's
        system at the current positions."""
        t = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.empty((max(len(t), 1), 4))
        self._check(self.lib.fdx_direct_forces(self.h, _ptr(t), len(t), float(eps), _ptr(out)),
                    "direct_forces")
        return out[:len(t)]

    # -- domain decomposition: multisection with cost-weighted sampling --------------------
    def decompose(self, nx: int, ny: int, nz: int, n_sample: int, cost=None, seed: int = 0,
                  cost_lists: bool = False):
        """cost: one value per current domain (system), or None (particle counts, or the
        list lengths of the last walk with cost_lists)."""
        cp = None
        if cost is not None:
            self._keep = [_f64(cost)]
            cp = _ptr(self._keep[0])
        self._check(self.lib.fdx_decompose(self.h, int(nx), int(ny), int(nz), int(n_sample), cp,
                                           int(seed) & (2 ** 64 - 1),
                                           DD_COST_LISTS if cost_lists else 0), "decompose")

    def dd_stats(self) -> dict:
        st = DdStats()
        self._check(self.lib.fdx_get_dd_stats(self.h, C.byref(st)), "get_dd_stats")
        return st.as_dict()

    def decomposition(self) -> dict:
        """faces bx [nx+1], by [nx, ny+1], bz [nx, ny, nz+1]; send counts [source, destination];
        dom_off [n_domains+1]."""
        st = self.dd_stats()
        nx, ny, nz, D, S = st["nx"], st["ny"], st["nz"], st["n_domains"], st["n_src"]
        bx, by, bz = np.empty(nx + 1), np.empty((nx, ny + 1)), np.empty((nx, ny, nz + 1))
        counts, off = np.empty((S, D), np.int64), np.empty(D + 1, np.int64)
        self._check(self.lib.fdx_get_decomposition(self.h, _ptr(bx), _ptr(by), _ptr(bz),
                                                   _ptr(counts), _ptr(off)), "get_decomposition")
        return {"bx": bx, "by": by, "bz": bz, "counts": counts, "dom_off": off}

    def dd_samples(self):
        """(k per current domain, particle index of every sample, domain of every sample)."""
        st = self.dd_stats()
        K = int(st["n_samples"])
        k = np.empty(st["n_src"], np.int64)
        idx, cell = np.empty(max(K, 1), np.uint32), np.empty(max(K, 1), np.uint32)
        self._check(self.lib.fdx_get_dd_samples(self.h, _ptr(k), _ptr(idx), _ptr(cell)),
                    "get_dd_samples")
        return k, idx[:K], cell[:K]

    def dd_destinations(self):
        """(dest per particle in the current order, order[r] = current index at new position r)
        as numpy arrays."""
        dest, order = np.empty(max(self.n, 1), np.uint32), np.empty(max(self.n, 1), np.uint32)
        self._check(self.lib.fdx_get_dd_destinations(self.h, _ptr(dest), _ptr(order), MEM_HOST),
                    "get_dd_destinations")
        return dest[:self.n], order[:self.n]

    def exchange_particles(self):
        self._check(self.lib.fdx_exchange_particles(self.h), "exchange_particles")

    # -- tree part of TreePM ----------------------------------------------------------------
    def calc_force_cutoff(self, theta: float, n_leaf: int, n_group: int, eps: float,
                          r_cut: float, fp32: bool = False, persistent: bool = False,
                          timing: bool = False):
        flags = ((FP32REL if fp32 else 0) | (PERSISTENT if persistent else 0)
                 | (TIMING if timing else 0))
        self._check(self.lib.fdx_calc_force_cutoff(self.h, float(theta), int(n_leaf),
                                                   int(n_group), float(eps), float(r_cut), flags),
                    "calc_force_cutoff")

    # -- short-range neighbour lists and SPH density -------------------------------------
    def calc_density(self, mode: int, r_cut: float = 0.0, h=None, n_leaf: int = 8,
                     n_group: int = 64, timing: bool = False):
        """h: per-particle support radius (numpy array, caller's order) or a device tensor."""
        hp, kind = None, MEM_HOST
        if h is not None:
            if hasattr(h, "data_ptr"):
                hp, kind = _dptr(h), MEM_DEVICE
                self._keep = [h]
            else:
                hh = _f64(h)
                self._keep = [hh]
                hp = _ptr(hh)
        self._check(self.lib.fdx_calc_density(self.h, int(mode), float(r_cut), hp, kind,
                                              int(n_leaf), int(n_group),
                                              TIMING if timing else 0), "calc_density")

    def density(self):
        """(rho, n_ngb) in the caller's order."""
        rho = np.empty(self.n)
        n = np.empty(self.n, np.uint32)
        self._check(self.lib.fdx_get_density(self.h, _ptr(rho), _ptr(n), MEM_HOST), "get_density")
        return rho, n

    # -- learned list-length predictor -----------------------------------------------------
    def predictor_features(self) -> np.ndarray:
        G = int(self.stats()["n_groups"])
        X = np.empty((max(G, 1), 8), np.float32)
        self._check(self.lib.fdx_predictor_features(self.h, _ptr(X)), "predictor_features")
        return X[:G]

    def mlp_forward(self, P, X) -> np.ndarray:
        P = np.ascontiguousarray(P, np.float32)
        X = np.ascontiguousarray(X, np.float32)
        y = np.empty(X.shape[0], np.float32)
        self._check(self.lib.fdx_mlp_forward(self.h, _ptr(P), _ptr(X), X.shape[0], _ptr(y)),
                    "mlp_forward")
        return y

    def mlp_grad(self, P, X, t):
        P = np.ascontiguousarray(P, np.float32)
        X = np.ascontiguousarray(X, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        g = np.empty(P.shape[0], np.float32)
        loss = np.zeros(1, np.float32)
        self._check(self.lib.fdx_mlp_grad(self.h, _ptr(P), _ptr(X), _ptr(t), X.shape[0], _ptr(g),
                                          _ptr(loss)), "mlp_grad")
        return g, float(loss[0])

    def mlp_adam(self, P, m, v, grads, step0=0, lr=1e-3):
        """Adam steps of the training kernel: returns the new (P, m, v) after one step per row
        of grads."""
        P, m, v = (np.array(a, np.float32) for a in (P, m, v))
        g = np.ascontiguousarray(grads, np.float32).reshape(-1, P.shape[0])
        self._check(self.lib.fdx_mlp_adam(self.h, _ptr(P), _ptr(m), _ptr(v), _ptr(g), g.shape[0],
                                          int(step0), float(lr)), "mlp_adam")
        return P, m, v

    def predictor_train(self, X, t, epochs=20, batch=4096, lr=1e-3, seed=1):
        X = np.ascontiguousarray(X, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        losses = np.zeros(epochs, np.float32)
        self._check(self.lib.fdx_predictor_train(self.h, _ptr(X), _ptr(t), X.shape[0], epochs,
                                                 batch, float(lr), int(seed), _ptr(losses)),
                    "predictor_train")
        return losses

    def predictor_margin(self, margin=float("nan")) -> float:
        out = C.c_double()
        self._check(self.lib.fdx_predictor_margin(self.h, float(margin), C.byref(out)),
                    "predictor_margin")
        return out.value

    def predictor_save(self, path: str):
        self._check(self.lib.fdx_predictor_save(self.h, path.encode()), "predictor_save")

    def predictor_load(self, path: str):
        self._check(self.lib.fdx_predictor_load(self.h, path.encode()), "predictor_load")


def calc_force_noalloc(device: int, stream, x, y, z, m, eps, eps_all: float, theta: float,
                       n_leaf: int, n_group: int, flags: int, ax, ay, az, pot):
    """fdx_calc_force_noalloc on device tensors (torch FP64, contiguous, one length); eps may
    be None.  stream: a torch stream or None (the null stream).  Raises FdxError on failure."""
    L = load()
    n = int(x.numel())
    s = None if stream is None else C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    err = C.create_string_buffer(256)
    rc = L.fdx_calc_force_noalloc(int(device), s, n, _dptr(x), _dptr(y), _dptr(z), _dptr(m),
                                  _dptr(eps), float(eps_all), float(theta), int(n_leaf),
                                  int(n_group), int(flags), _dptr(ax), _dptr(ay), _dptr(az),
                                  _dptr(pot), err, 256)
    if rc != OK:
        raise FdxError(rc, f"calc_force_noalloc: {err.value.decode()}")


def dd_factor(n: int):
    """(n_x, n_y, n_z) for n domains, integers close to n^(1/3)."""
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    r = load().fdx_dd_factor(int(n), C.byref(a), C.byref(b), C.byref(c))
    if r != 0:
        raise FdxError(r, "dd_factor: n must be >= 1")
    return a.value, b.value, c.value
