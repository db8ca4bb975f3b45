"""Batched sweeps: many independent sLdG problems advanced together.

ctypes binding of the sldg_batch_* entry points (include/sldg.h).  Each sweep
of a split step is one work list of tiles over every problem, launched as one
kernel per class (tile kind x degree, each class compiled for itself); a step
can be captured into a HIP graph and replayed; the launch shape of every
class is tuned on the bound data, and tuned shapes can be stored in a JSON
cache keyed by the batch's shape signature.  Marshalling only: every step runs
in the library's kernels.
"""
import ctypes
import hashlib
import json
import os

from . import _check, _current_stream, _ptr, hi_dtype, lib, TIERS, TIER_BYTES

_bound = False


def _lib():
    global _bound
    L = lib()
    if not _bound:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.sldg_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(i64),
                                        ctypes.POINTER(i32), i32, vp]
        L.sldg_batch_create.restype = i32
        L.sldg_batch_destroy.argtypes = [vp]
        L.sldg_batch_destroy.restype = None
        L.sldg_batch_bind.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.sldg_batch_bind.restype = i32
        L.sldg_batch_set_sequence.argtypes = [vp, i32, ctypes.POINTER(i32),
                                              ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(vp)]
        L.sldg_batch_set_sequence.restype = i32
        L.sldg_batch_run.argtypes = [vp, i32, i32, ctypes.POINTER(i32)]
        L.sldg_batch_run.restype = i32
        L.sldg_batch_tune.argtypes = [vp, i32]
        L.sldg_batch_tune.restype = i32
        L.sldg_batch_get_tuning.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(ctypes.c_double)]
        L.sldg_batch_get_tuning.restype = i32
        L.sldg_batch_set_tuning.argtypes = [vp, i32, i32, i32]
        L.sldg_batch_set_tuning.restype = i32
        L.sldg_batch_get_class_tuning.argtypes = [vp, i32, i32, ctypes.POINTER(i32),
                                                  ctypes.POINTER(i32),
                                                  ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(i32)]
        L.sldg_batch_get_class_tuning.restype = i32
        L.sldg_batch_set_class_tuning.argtypes = [vp, i32, i32, i32, i32]
        L.sldg_batch_set_class_tuning.restype = i32
        _bound = True
    return L


class Batch:
    """Problems with extents `ncells[p]` (tuples, dimension 0 fastest, same
    dimension count) and degrees `ks[p]`, one storage tier."""

    def __init__(self, ncells, ks, tier="fp32", stream=None):
        self.ncells = [tuple(int(v) for v in n) for n in ncells]
        self.ks = [int(k) for k in ks]
        self.nprob = len(self.ncells)
        if self.nprob != len(self.ks) or self.nprob == 0:
            raise ValueError("need one degree per problem and at least one problem")
        self.ndim = len(self.ncells[0])
        if any(len(n) != self.ndim for n in self.ncells):
            raise ValueError("every problem of a batch has the same dimension count")
        if tier not in TIERS:
            raise ValueError(f"unknown tier {tier!r}")
        self.tier = tier
        self.cells = [1] * self.nprob
        for p, n in enumerate(self.ncells):
            for v in n:
                self.cells[p] *= v
        self.modes = [(k + 1) ** self.ndim for k in self.ks]
        self.stream = _current_stream() if stream is None else stream
        flat = [v for n in self.ncells for v in n]
        h = ctypes.c_void_p()
        _check(_lib().sldg_batch_create(ctypes.byref(h), self.nprob, self.ndim,
                                        (ctypes.c_int64 * len(flat))(*flat),
                                        (ctypes.c_int * self.nprob)(*self.ks), TIERS[tier],
                                        ctypes.c_void_p(self.stream)), "sldg_batch_create")
        self._h = h
        self._states = None
        self.nseq = 0

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("batch destroyed")
        return self._h

    def signature(self):
        """Shape signature (problems, degrees, tier, sequence dims) for tuning caches."""
        txt = json.dumps([self.ncells, self.ks, self.tier, getattr(self, "_dims", [])])
        return hashlib.sha256(txt.encode()).hexdigest()[:24]

    def empty_states(self, device="cuda"):
        """Two lists of (mass, hi) device tensors, one pair per problem."""
        import torch
        out = []
        for _ in range(2):
            st = []
            for p in range(self.nprob):
                st.append((torch.empty(self.cells[p], dtype=torch.float64, device=device),
                           torch.empty((self.modes[p] - 1, self.cells[p]),
                                       dtype=hi_dtype(self.tier), device=device)))
            out.append(st)
        return out

    def bind(self, states0, states1):
        """Bind buffer 0 and buffer 1 of every problem (lists of (mass, hi))."""
        import torch
        for states in (states0, states1):
            if len(states) != self.nprob:
                raise ValueError("one (mass, hi) pair per problem")
            for p, (m, h) in enumerate(states):
                if not (isinstance(m, torch.Tensor) and isinstance(h, torch.Tensor)) or \
                        not (m.is_cuda and h.is_cuda):
                    raise ValueError("state buffers must be device tensors")
                if m.dtype != torch.float64 or not m.is_contiguous() or m.numel() < self.cells[p]:
                    raise ValueError(f"problem {p}: bad mass buffer")
                need = (self.modes[p] - 1) * self.cells[p] * TIER_BYTES[self.tier]
                if h.dtype != hi_dtype(self.tier) or not h.is_contiguous() or \
                        h.numel() * h.element_size() < need:
                    raise ValueError(f"problem {p}: bad hi buffer")
        arr = lambda xs: (ctypes.c_void_p * self.nprob)(*[_ptr(x) for x in xs])
        _check(_lib().sldg_batch_bind(self.handle, arr([s[0] for s in states0]),
                                      arr([s[1] for s in states0]), arr([s[0] for s in states1]),
                                      arr([s[1] for s in states1])), "sldg_batch_bind")
        self._states = (states0, states1)

    def set_sequence(self, seq):
        """seq: list of (dim, [(dep_mask, shift tensor) for every problem])."""
        import torch
        nseq = len(seq)
        dims = (ctypes.c_int * nseq)(*[int(d) for d, _ in seq])
        masks = (ctypes.c_uint32 * (nseq * self.nprob))()
        ptrs = (ctypes.c_void_p * (nseq * self.nprob))()
        keep = []
        for q, (dim, per) in enumerate(seq):
            if len(per) != self.nprob:
                raise ValueError("one (mask, shift) per problem")
            for p, (mask, shift) in enumerate(per):
                need = 1
                for e in range(self.ndim):
                    if mask >> e & 1:
                        need *= self.ncells[p][e]
                if not isinstance(shift, torch.Tensor) or not shift.is_cuda or \
                        shift.dtype != torch.float64 or not shift.is_contiguous() or \
                        shift.numel() < need:
                    raise ValueError(f"sweep {q} problem {p}: shift must be a float64 device "
                                     f"tensor of >= {need} elements")
                masks[q * self.nprob + p] = int(mask)
                ptrs[q * self.nprob + p] = _ptr(shift)
                keep.append(shift)
        _check(_lib().sldg_batch_set_sequence(self.handle, nseq, dims, masks, ptrs),
               "sldg_batch_set_sequence")
        self.nseq = nseq
        self._dims = [int(d) for d, _ in seq]
        self._shifts = keep

    def run(self, nsteps, use_graph=False):
        """nsteps split steps; returns the buffer index holding the result."""
        res = ctypes.c_int(-1)
        _check(_lib().sldg_batch_run(self.handle, int(nsteps), 1 if use_graph else 0,
                                     ctypes.byref(res)), "sldg_batch_run")
        return res.value

    def tune(self, reps=3):
        """Time the launch shapes of every sweep and keep the fastest (clobbers buffer 1)."""
        _check(_lib().sldg_batch_tune(self.handle, int(reps)), "sldg_batch_tune")
        return self.tuning()

    CLASSES = 9         # work-list classes: 3 * kind + k - 1 (kind 0 window, 1 group, 2 strided)

    def tuning(self):
        """Per sweep: the shape of its largest class, the tuned time of the
        sweep, and the shape, time and tile count of every non-empty class."""
        out = []
        for q in range(self.nseq):
            r, t, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
            _check(_lib().sldg_batch_get_tuning(self.handle, q, ctypes.byref(r), ctypes.byref(t),
                                                ctypes.byref(ms)), "sldg_batch_get_tuning")
            classes = {}
            for c in range(self.CLASSES):
                cr, ct, cms, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
                _check(_lib().sldg_batch_get_class_tuning(self.handle, q, c, ctypes.byref(cr),
                                                          ctypes.byref(ct), ctypes.byref(cms),
                                                          ctypes.byref(n)),
                       "sldg_batch_get_class_tuning")
                if n.value:
                    classes[str(c)] = {"rows": cr.value, "tuples": ct.value, "ms": cms.value,
                                       "tiles": n.value}
            out.append({"rows": r.value, "tuples": t.value, "ms": ms.value, "classes": classes})
        return out

    def set_class_tuning(self, q, cls, rows, tuples):
        """Launch shape of class `cls` of sweep q alone
        (sldg_batch_set_class_tuning)."""
        _check(_lib().sldg_batch_set_class_tuning(self.handle, int(q), int(cls), int(rows),
                                                  int(tuples)), "sldg_batch_set_class_tuning")

    def set_tuning(self, shapes):
        """Apply shapes as `tuning()` returns them (per class when given)."""
        for q, sh in enumerate(shapes):
            _check(_lib().sldg_batch_set_tuning(self.handle, q, int(sh["rows"]), int(sh["tuples"])),
                   "sldg_batch_set_tuning")
            for c, cs in sh.get("classes", {}).items():
                _check(_lib().sldg_batch_set_class_tuning(self.handle, q, int(c), int(cs["rows"]),
                                                          int(cs["tuples"])),
                       "sldg_batch_set_class_tuning")

    def tune_cached(self, path, reps=3):
        """Tuned shapes from the JSON cache at `path` if it has this batch's
        signature, else tune now and store them."""
        cache = {}
        if os.path.exists(path):
            with open(path) as f:
                cache = json.load(f)
        key = self.signature()
        if key in cache:
            self.set_tuning(cache[key])
            return cache[key], True
        shapes = self.tune(reps)
        cache[key] = shapes
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
        return shapes, False

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib().sldg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
