"""paper_1910_03936_amd: MI355X-native pre-alignment filtering (SneakySnake,
GateKeeper, Shouji) after Alser's thesis (arXiv 1910.03936).

This module is a thin ctypes binding over libpaf.so (include/paf.h): it only
marshals PyTorch device tensors and streams into the C ABI.  Every step of the
filter runs in the library's HIP kernels; there is no CPU fallback, and
importing the binding fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaf.so")

SNEAKYSNAKE, GATEKEEPER, SHOUJI = 1, 2, 4
ALL_FILTERS = SNEAKYSNAKE | GATEKEEPER | SHOUJI
MAX_LEN, MAX_E = 512, 31
MAX_PART = 65535  # widest sub-maze of paf_filter_partitioned
MAX_REPL = 31     # most replications (obstacles per sub-maze) of paf_filter_partitioned
MAGNET_NOALLOC_MAX_PAIRS = 4194304   # largest batch of paf_filter_magnet_noalloc
MLP_NPARAMS = 24961
STATE_MAGIC, STATE_VERSION = 0x46415053, 1   # "SPAF": files written by Context.save_state

STATUS = {0: "PAF_OK", 1: "PAF_ERR_ARG", 2: "PAF_ERR_RANGE", 3: "PAF_ERR_DEVICE",
          4: "PAF_ERR_NOMEM", 5: "PAF_ERR_STATE"}

# Every symbol declared in include/paf.h.
EXPORTS = ("paf_create", "paf_destroy", "paf_last_error", "paf_check", "paf_pack", "paf_pack_host", "paf_pack_ascii",
           "paf_filter", "paf_filter_partitioned", "paf_filter_magnet", "paf_filter_magnet_noalloc", "paf_verify",
           "paf_filter_persistent", "paf_autotune", "paf_set_layout", "paf_tuned_export", "paf_tuned_import",
           "paf_features", "paf_mlp_set_params", "paf_mlp_get_params", "paf_mlp_get_state", "paf_mlp_set_state",
           "paf_mlp_forward", "paf_mlp_train_step", "paf_mlp_predict", "paf_mlp_train", "paf_bucket",
           "paf_filter_ordered", "paf_filter_bucketed", "paf_filter_bucketed_local", "paf_cost_levels",
           "paf_filter_keyed", "paf_stream_filter")


class PafError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Batch(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_void_p), ("refs", ctypes.c_void_p),
                ("word_offset", ctypes.c_void_p), ("stride_words", ctypes.c_uint32),
                ("len", ctypes.c_void_p), ("uniform_len", ctypes.c_uint16),
                ("E", ctypes.c_void_p), ("uniform_E", ctypes.c_uint8),
                ("max_len", ctypes.c_uint16), ("max_E", ctypes.c_uint8),
                ("n_pairs", ctypes.c_uint64)]


class _Out(ctypes.Structure):
    _fields_ = [("accept_bits", ctypes.c_void_p * 3), ("count", ctypes.c_void_p * 3)]


class _HostBatch(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_void_p), ("refs", ctypes.c_void_p), ("len", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("max_len", ctypes.c_uint16), ("max_E", ctypes.c_uint8),
                ("n_pairs", ctypes.c_uint64)]


class _StreamStats(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("h2d_bytes", ctypes.c_double), ("chunks", ctypes.c_uint64)]


class Layout(ctypes.Structure):
    _fields_ = [("lanes_per_pair", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("tiles_per_grab", ctypes.c_uint32),
                ("chunk_tiles", ctypes.c_uint32), ("first_pass_windows", ctypes.c_uint32),
                ("pass_windows", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class _TunedEntry(ctypes.Structure):
    _fields_ = [("max_words", ctypes.c_uint32), ("max_E", ctypes.c_uint32), ("filters", ctypes.c_uint32),
                ("layout", Layout)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpaf.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpaf.so not built at {path}: run __graft_entry__.build() "
                          f"or python -m paper_1910_03936_amd.build")
    lib = ctypes.CDLL(path)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "paf_create": ([ctypes.POINTER(P), I]),
        "paf_destroy": ([P]),
        "paf_check": ([P, P]),
        "paf_pack": ([P, P, U32, P, ctypes.c_uint16, P, U32, U64, P, P]),
        "paf_pack_host": ([P, U32, P, ctypes.c_uint16, P, U32, U64, P, I]),
        "paf_pack_ascii": ([P, U32, P, ctypes.c_uint16, P, U32, U64, P, I]),
        "paf_filter": ([P, ctypes.POINTER(_Batch), U32, ctypes.POINTER(_Out), P]),
        "paf_filter_persistent": ([P, ctypes.POINTER(_Batch), U32, ctypes.POINTER(_Out), P]),
        "paf_filter_partitioned": ([P, ctypes.POINTER(_Batch), U32, U32, ctypes.POINTER(_Out), P]),
        "paf_verify": ([P, ctypes.POINTER(_Batch), P, P, P]),
        "paf_filter_magnet": ([P, ctypes.POINTER(_Batch), ctypes.POINTER(_Out), P]),
        "paf_filter_magnet_noalloc": ([P, ctypes.POINTER(_Batch), ctypes.POINTER(_Out), P]),
        "paf_autotune": ([P, ctypes.POINTER(_Batch), U32, ctypes.POINTER(_Out), P,
                          ctypes.POINTER(Layout), ctypes.POINTER(ctypes.c_float),
                          ctypes.POINTER(ctypes.c_float)]),
        "paf_set_layout": ([P, ctypes.POINTER(Layout)]),
        "paf_tuned_export": ([P, ctypes.POINTER(_TunedEntry), U32, ctypes.POINTER(U32)]),
        "paf_tuned_import": ([P, ctypes.POINTER(_TunedEntry), U32]),
        "paf_mlp_get_state": ([P, P, P, P, ctypes.POINTER(U32)]),
        "paf_mlp_set_state": ([P, P, P, P, U32]),
        "paf_features": ([P, ctypes.POINTER(_Batch), P, P]),
        "paf_mlp_set_params": ([P, P]),
        "paf_mlp_get_params": ([P, P]),
        "paf_mlp_forward": ([P, P, U64, P, P]),
        "paf_mlp_train_step": ([P, P, P, U64, ctypes.c_float, P, P, P]),
        "paf_bucket": ([P, ctypes.POINTER(_Batch), P, P, P, P]),
        "paf_mlp_predict": ([P, ctypes.POINTER(_Batch), P, P]),
        "paf_mlp_train": ([P, P, P, U64, U32, U32, ctypes.c_float, P, P]),
        "paf_filter_bucketed": ([P, ctypes.POINTER(_Batch), U32, ctypes.POINTER(_Out), P]),
        "paf_filter_bucketed_local": ([P, ctypes.POINTER(_Batch), ctypes.POINTER(_Out), P]),
        "paf_cost_levels": ([P, ctypes.POINTER(_Batch), P, P]),
        "paf_filter_keyed": ([P, ctypes.POINTER(_Batch), P, ctypes.POINTER(_Out), P]),
        "paf_filter_ordered": ([P, ctypes.POINTER(_Batch), U32, P, ctypes.POINTER(_Out), P]),
        "paf_stream_filter": ([P, ctypes.POINTER(_HostBatch), U64, U32, I, ctypes.POINTER(_Out),
                               ctypes.POINTER(_StreamStats)]),
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.paf_last_error.argtypes = []
    lib.paf_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = _lib.paf_last_error().decode(errors="replace")
        raise PafError(status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def pack_ascii(seqs, threads: int = 0):
    """Encode equal-length DNA strings (A/C/G/T, either case) into the planar
    two-bit words of paf.h on the host (paf_pack_ascii): returns a numpy uint64
    array of len(seqs) * ceil(m / 32) words, the rows back to back.  Raises
    PafError (PAF_ERR_ARG) on any other letter."""
    import numpy as np

    load_library()
    if not seqs:
        raise ValueError("no sequences")
    m = len(seqs[0])
    if any(len(x) != m for x in seqs):
        raise ValueError("sequences differ in length")
    rows = np.frombuffer("".join(seqs).encode("latin-1"), dtype=np.uint8)
    W = words_for(m)
    out = np.zeros(len(seqs) * W, np.uint64)
    _check(_lib.paf_pack_ascii(rows.ctypes.data_as(ctypes.c_void_p), m, None, m, None, W, len(seqs),
                               out.ctypes.data_as(ctypes.c_void_p), threads))
    return out


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def words_for(m: int) -> int:
    return (m + 31) // 32


@dataclass
class Batch:
    """Device-resident packed pairs, in the layout of paf_batch."""
    reads: torch.Tensor                      # int64 words (uint64 bit patterns)
    refs: torch.Tensor
    n_pairs: int
    stride_words: int = 0
    word_offset: torch.Tensor | None = None  # int64 [n]
    len: torch.Tensor | None = None          # int16 [n] (uint16 values)
    E: torch.Tensor | None = None            # uint8 [n]
    uniform_len: int = 0
    uniform_E: int = 0
    max_len: int = 0
    max_E: int = 0

    def c(self) -> _Batch:
        b = _Batch()
        b.reads = self.reads.data_ptr()
        b.refs = self.refs.data_ptr()
        b.word_offset = None if self.word_offset is None else self.word_offset.data_ptr()
        b.stride_words = self.stride_words
        b.len = None if self.len is None else self.len.data_ptr()
        b.uniform_len = self.uniform_len
        b.E = None if self.E is None else self.E.data_ptr()
        b.uniform_E = self.uniform_E
        b.max_len = self.max_len or self.uniform_len
        b.max_E = self.max_E or self.uniform_E
        b.n_pairs = self.n_pairs
        return b

    @property
    def device(self):
        return self.reads.device


class Context:
    """Owns a paf_ctx on one device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.paf_create(ctypes.byref(h), device))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(self.lib.paf_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, stream=None):
        _check(self.lib.paf_check(self.h, _stream(stream)))

    # -- encode -------------------------------------------------------------
    def pack(self, codes: torch.Tensor, lens: torch.Tensor | None = None, uniform_len: int = 0,
             word_offset: torch.Tensor | None = None, stride_words: int = 0, total_words: int = 0,
             stream=None) -> torch.Tensor:
        """codes: uint8 [n, code_stride] device tensor -> int64 words."""
        n, cs = codes.shape
        if word_offset is None:
            stride_words = stride_words or words_for(uniform_len or cs)
            total_words = n * stride_words
        words = torch.zeros(max(total_words, 1), dtype=torch.int64, device=codes.device)
        _check(self.lib.paf_pack(self.h, _ptr(codes), cs, _ptr(lens), uniform_len, _ptr(word_offset),
                                 stride_words, n, _ptr(words), _stream(stream)))
        return words

    def pack_pairs(self, reads_u8: torch.Tensor, refs_u8: torch.Tensor, lens=None, Es=None,
                   uniform_len: int = 0, uniform_E: int = 0, max_len: int = 0, max_E: int = 0,
                   offsets: bool = False, stream=None) -> Batch:
        """Pack a batch of uint8 pairs (device tensors [n, stride]) into a Batch.
        offsets=True packs per-pair lengths compactly with word offsets."""
        n, cs = reads_u8.shape
        dev = reads_u8.device
        if lens is not None and offsets:
            w = (lens.to(torch.int64) + 31) // 32
            off = torch.zeros(n, dtype=torch.int64, device=dev)
            off[1:] = torch.cumsum(w, 0)[:-1]
            total = int(w.sum().item())
            rd = self.pack(reads_u8, lens, 0, off, 0, total, stream)
            rf = self.pack(refs_u8, lens, 0, off, 0, total, stream)
            return Batch(rd, rf, n, 0, off, lens, Es, 0, uniform_E, max_len or cs, max_E or uniform_E)
        stride = words_for(max_len or uniform_len or cs)
        rd = self.pack(reads_u8, lens, uniform_len, None, stride, 0, stream)
        rf = self.pack(refs_u8, lens, uniform_len, None, stride, 0, stream)
        return Batch(rd, rf, n, stride, None, lens, Es, uniform_len, uniform_E,
                     max_len or uniform_len or cs, max_E or uniform_E)

    # -- filter ---------------------------------------------------------
    def alloc_out(self, n: int, filters: int, device) -> dict:
        out = {}
        for f in range(3):
            if filters & (1 << f):
                out[1 << f] = (torch.zeros((n + 31) // 32, dtype=torch.int32, device=device),
                               torch.zeros(n, dtype=torch.int16, device=device))
        return out

    @staticmethod
    def _out(out: dict) -> _Out:
        o = _Out()
        for f in range(3):
            if (1 << f) in out:
                a, c = out[1 << f]
                o.accept_bits[f] = a.data_ptr()
                o.count[f] = c.data_ptr()
        return o

    def filter(self, batch: Batch, filters: int = SNEAKYSNAKE, out: dict | None = None,
               stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, filters, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter(self.h, ctypes.byref(cb), filters, ctypes.byref(co), _stream(stream)))
        return out

    def filter_partitioned(self, batch: Batch, t: int, y: int = 0, out: dict | None = None, stream=None) -> dict:
        """SneakySnake on the maze cut into sub-mazes of t columns; y > 0: at
        most y obstacles per sub-maze (the hardware form's y replications)."""
        out = out or self.alloc_out(batch.n_pairs, SNEAKYSNAKE, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_partitioned(self.h, ctypes.byref(cb), t, y, ctypes.byref(co),
                                               _stream(stream)))
        return out

    def filter_magnet(self, batch: Batch, out: dict | None = None, stream=None) -> dict:
        """MAGNET's decision (accept bits and count in the SneakySnake slot)."""
        out = out or self.alloc_out(batch.n_pairs, SNEAKYSNAKE, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_magnet(self.h, ctypes.byref(cb), ctypes.byref(co), _stream(stream)))
        return out

    def verify(self, batch: Batch, select_bits: torch.Tensor | None = None, dist: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
        """min(banded edit distance, E + 1) per pair (int16 storage of uint16);
        with select_bits (accept-bit words) only the selected pairs are
        verified and the others get E + 1."""
        if dist is None:
            dist = torch.empty(batch.n_pairs, dtype=torch.int16, device=batch.device)
        cb = batch.c()
        sel = None if select_bits is None else _ptr(select_bits)
        _check(self.lib.paf_verify(self.h, ctypes.byref(cb), sel, _ptr(dist), _stream(stream)))
        return dist

    def filter_persistent(self, batch: Batch, filters: int = SNEAKYSNAKE, out: dict | None = None,
                          stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, filters, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_persistent(self.h, ctypes.byref(cb), filters, ctypes.byref(co),
                                              _stream(stream)))
        return out

    def autotune(self, batch: Batch, filters: int = SNEAKYSNAKE, stream=None):
        out = self.alloc_out(batch.n_pairs, filters, batch.device)
        cb, co = batch.c(), self._out(out)
        lay = Layout()
        best, dflt = ctypes.c_float(), ctypes.c_float()
        _check(self.lib.paf_autotune(self.h, ctypes.byref(cb), filters, ctypes.byref(co), _stream(stream),
                                     ctypes.byref(lay), ctypes.byref(best), ctypes.byref(dflt)))
        return lay.as_dict(), best.value, dflt.value

    def set_layout(self, layout: dict | None):
        if layout is None:
            _check(self.lib.paf_set_layout(self.h, None))
        else:
            lay = Layout(**layout)
            _check(self.lib.paf_set_layout(self.h, ctypes.byref(lay)))

    # -- checkpoint / resume -------------------------------------------
    def tuned_export(self) -> list:
        """The autotuner's cache: [{"max_words", "max_E", "filters", "layout": {...}}]."""
        n = ctypes.c_uint32()
        _check(self.lib.paf_tuned_export(self.h, None, 0, ctypes.byref(n)))
        arr = (_TunedEntry * max(1, n.value))()
        _check(self.lib.paf_tuned_export(self.h, arr, n.value, ctypes.byref(n)))
        return [{"max_words": int(e.max_words), "max_E": int(e.max_E), "filters": int(e.filters),
                 "layout": e.layout.as_dict()} for e in arr[:n.value]]

    def tuned_import(self, entries: list):
        arr = (_TunedEntry * max(1, len(entries)))()
        for i, e in enumerate(entries):
            arr[i] = _TunedEntry(e["max_words"], e["max_E"], e["filters"], Layout(**e["layout"]))
        _check(self.lib.paf_tuned_import(self.h, arr, len(entries)))

    def mlp_get_state(self) -> dict:
        import numpy as np
        st = {k: np.zeros(MLP_NPARAMS, np.float32) for k in ("params", "adam_m", "adam_v")}
        step = ctypes.c_uint32()
        _check(self.lib.paf_mlp_get_state(self.h, *(st[k].ctypes.data_as(ctypes.c_void_p)
                                                    for k in ("params", "adam_m", "adam_v")), ctypes.byref(step)))
        st["step"] = int(step.value)
        return st

    def mlp_set_state(self, st: dict):
        import numpy as np
        a = {k: np.ascontiguousarray(np.asarray(st[k], dtype=np.float32)) for k in ("params", "adam_m", "adam_v")}
        for k, v in a.items():
            if v.shape != (MLP_NPARAMS,):
                raise ValueError(f"{k} has shape {v.shape}, expected ({MLP_NPARAMS},)")
        _check(self.lib.paf_mlp_set_state(self.h, *(a[k].ctypes.data_as(ctypes.c_void_p)
                                                    for k in ("params", "adam_m", "adam_v")), int(st["step"])))

    def save_state(self, path: str, model: bool = True):
        """Writes the autotune cache and (if `model` and one is loaded) the cost
        model with its optimizer state to one .npz file (plain arrays, no
        pickled objects)."""
        import numpy as np
        tuned = self.tuned_export()
        rows = np.array([[e["max_words"], e["max_E"], e["filters"]] + [e["layout"][f] for f, _ in Layout._fields_]
                         for e in tuned], dtype=np.uint32).reshape(len(tuned), 3 + len(Layout._fields_))
        arrays = {"format": np.array([STATE_MAGIC, STATE_VERSION], dtype=np.uint32), "tuned": rows}
        if model:
            try:
                st = self.mlp_get_state()
            except PafError as e:
                if e.status != 5:   # PAF_ERR_STATE: no model to save
                    raise
            else:
                arrays.update(mlp_params=st["params"], adam_m=st["adam_m"], adam_v=st["adam_v"],
                              adam_step=np.array([st["step"]], dtype=np.uint32))
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    def load_state(self, path: str) -> dict:
        """Reads a file written by save_state and applies it (the library checks
        every value first).  Returns what was loaded: {"tuned": n, "model": bool}."""
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            fmt = z["format"]
            if fmt.shape != (2,) or int(fmt[0]) != STATE_MAGIC or int(fmt[1]) != STATE_VERSION:
                raise ValueError(f"{path}: not a state file of this library (format {fmt.tolist()})")
            rows = z["tuned"]
            if rows.ndim != 2 or rows.shape[1] != 3 + len(Layout._fields_):
                raise ValueError(f"{path}: tuned table has shape {rows.shape}")
            entries = [{"max_words": int(r[0]), "max_E": int(r[1]), "filters": int(r[2]),
                        "layout": {f: int(v) for (f, _), v in zip(Layout._fields_, r[3:])}} for r in rows]
            st = None
            if "mlp_params" in z.files:
                st = {"params": z["mlp_params"], "adam_m": z["adam_m"], "adam_v": z["adam_v"],
                      "step": int(z["adam_step"][0])}
        self.tuned_import(entries)
        if st is not None:
            self.mlp_set_state(st)
        return {"tuned": len(entries), "model": st is not None}

    # -- cost model --------------------------------------------------
    def features(self, batch: Batch, stream=None) -> torch.Tensor:
        f = torch.empty((batch.n_pairs, 64), dtype=torch.float32, device=batch.device)
        cb = batch.c()
        _check(self.lib.paf_features(self.h, ctypes.byref(cb), _ptr(f), _stream(stream)))
        return f

    def mlp_set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        assert p.shape == (MLP_NPARAMS,)
        _check(self.lib.paf_mlp_set_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))

    def mlp_get_params(self):
        import numpy as np
        p = np.zeros(MLP_NPARAMS, np.float32)
        _check(self.lib.paf_mlp_get_params(self.h, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def mlp_forward(self, feats: torch.Tensor, stream=None) -> torch.Tensor:
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        _check(self.lib.paf_mlp_forward(self.h, _ptr(feats), feats.shape[0], _ptr(out), _stream(stream)))
        return out

    def mlp_train_step(self, feats: torch.Tensor, targets: torch.Tensor, lr: float,
                       want_grads: bool = False, stream=None):
        grads = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=feats.device) if want_grads else None
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        _check(self.lib.paf_mlp_train_step(self.h, _ptr(feats), _ptr(targets), feats.shape[0],
                                           ctypes.c_float(lr), _ptr(grads), _ptr(loss), _stream(stream)))
        return loss, grads

    def mlp_predict(self, batch: Batch, stream=None) -> torch.Tensor:
        """Fused features + model predictions for every pair of the batch."""
        pred = torch.empty(batch.n_pairs, dtype=torch.float32, device=batch.device)
        cb = batch.c()
        _check(self.lib.paf_mlp_predict(self.h, ctypes.byref(cb), _ptr(pred), _stream(stream)))
        return pred

    def mlp_train(self, feats: torch.Tensor, labels: torch.Tensor, epochs: int, batch: int, lr: float,
                  stream=None):
        """Train on feature rows [n][64] fp32 and uint16 labels (int16 tensor)."""
        import numpy as np
        loss = np.zeros(epochs, np.float32)
        _check(self.lib.paf_mlp_train(self.h, _ptr(feats), _ptr(labels), feats.shape[0], epochs, batch,
                                      ctypes.c_float(lr), loss.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return loss

    def bucket(self, batch: Batch, pred: torch.Tensor, stream=None):
        perm = torch.empty(batch.n_pairs, dtype=torch.int32, device=batch.device)
        hist = torch.empty(16, dtype=torch.int32, device=batch.device)
        cb = batch.c()
        _check(self.lib.paf_bucket(self.h, ctypes.byref(cb), _ptr(pred), _ptr(perm), _ptr(hist),
                                   _stream(stream)))
        return perm, hist

    def filter_ordered(self, batch: Batch, order: torch.Tensor, filters: int = SNEAKYSNAKE,
                       out: dict | None = None, stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, filters, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_ordered(self.h, ctypes.byref(cb), filters, _ptr(order), ctypes.byref(co),
                                           _stream(stream)))
        return out

    def cost_levels(self, batch: Batch, stream=None) -> torch.Tensor:
        """uint8 key per pair: 15 - the model's cost level (chunk-local order)."""
        key = torch.empty(batch.n_pairs, dtype=torch.uint8, device=batch.device)
        cb = batch.c()
        _check(self.lib.paf_cost_levels(self.h, ctypes.byref(cb), _ptr(key), _stream(stream)))
        return key

    def filter_keyed(self, batch: Batch, key: torch.Tensor, out: dict | None = None, stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, SNEAKYSNAKE, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_keyed(self.h, ctypes.byref(cb), _ptr(key), ctypes.byref(co), _stream(stream)))
        return out

    def filter_bucketed_local(self, batch: Batch, out: dict | None = None, stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, SNEAKYSNAKE, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_bucketed_local(self.h, ctypes.byref(cb), ctypes.byref(co), _stream(stream)))
        return out

    def filter_bucketed(self, batch: Batch, filters: int = SNEAKYSNAKE, out: dict | None = None,
                        stream=None) -> dict:
        out = out or self.alloc_out(batch.n_pairs, filters, batch.device)
        cb, co = batch.c(), self._out(out)
        _check(self.lib.paf_filter_bucketed(self.h, ctypes.byref(cb), filters, ctypes.byref(co),
                                            _stream(stream)))
        return out


@dataclass
class HostBatch:
    """Pairs in (pinned) host memory, stored back to back (see paf_host_batch)."""
    reads: torch.Tensor   # int64 words, CPU
    refs: torch.Tensor
    len: torch.Tensor     # int16, CPU
    E: torch.Tensor       # uint8, CPU
    max_len: int
    max_E: int

    @property
    def n_pairs(self) -> int:
        return int(self.len.shape[0])


def stream_filter(ctx: Context, hb: HostBatch, chunk_pairs: int, filters: int = SNEAKYSNAKE,
                  learned: bool = False, first_pair: int = 0, out: dict | None = None):
    """paf_stream_filter: returns ({filter: (accept bit words, counts)} in pinned
    host tensors, stats dict).

    Resume: the stream's progress is its chunk index, and filtering a chunk
    again writes the same outputs.  A stream stopped after c chunks resumes
    with first_pair = c * chunk_pairs and the `out` of the stopped call: only
    pairs first_pair.. are filtered (their words start after the first
    first_pair pairs' ceil(len / 32) words) and written into `out`."""
    n = hb.n_pairs
    if first_pair < 0 or first_pair > n or first_pair % 64 != 0:
        raise ValueError(f"first_pair {first_pair} must be a multiple of 64 in [0, {n}]")
    if out is None:
        out = {}
        for f in range(3):
            if filters & (1 << f):
                out[1 << f] = (torch.zeros((n + 31) // 32, dtype=torch.int32, pin_memory=True),
                               torch.zeros(n, dtype=torch.int16, pin_memory=True))
    o = _Out()
    for f in range(3):
        if filters & (1 << f):
            a, c = out[1 << f]
            if a.numel() * 32 < n or c.numel() < n:
                raise ValueError("out tensors are smaller than the batch")
            o.accept_bits[f] = a.data_ptr() + (first_pair // 32) * 4
            o.count[f] = c.data_ptr() + first_pair * 2
    if first_pair == n:
        return out, {"seconds": 0.0, "h2d_bytes": 0.0, "chunks": 0}
    w0 = int(((hb.len[:first_pair].to(torch.int64) + 31) // 32).sum()) if first_pair else 0
    b = _HostBatch(hb.reads.data_ptr() + 8 * w0, hb.refs.data_ptr() + 8 * w0, hb.len.data_ptr() + 2 * first_pair,
                   hb.E.data_ptr() + first_pair, hb.max_len, hb.max_E, n - first_pair)
    st = _StreamStats()
    _check(ctx.lib.paf_stream_filter(ctx.h, ctypes.byref(b), chunk_pairs, filters, int(learned),
                                     ctypes.byref(o), ctypes.byref(st)))
    return out, {"seconds": st.seconds, "h2d_bytes": st.h2d_bytes, "chunks": int(st.chunks)}


def accept_bits_to_bool(bits: torch.Tensor, n: int) -> torch.Tensor:
    """Unpack accept-bit words (bit p%32 of word p/32) into a bool tensor [n]."""
    b = bits.to(torch.int64) & 0xFFFFFFFF
    shifts = torch.arange(32, device=bits.device, dtype=torch.int64)
    return ((b[:, None] >> shifts[None, :]) & 1).reshape(-1)[:n].bool()


def counts_u16(c: torch.Tensor) -> torch.Tensor:
    """int16 storage of uint16 counts -> int32 values."""
    return c.to(torch.int32) & 0xFFFF
