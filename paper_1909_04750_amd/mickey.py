"""ctypes binding of libmickey.so (include/mickey.h, include/grain.h, include/aes.h).  Argument marshalling only: every
step of the keystream path runs in the library's HIP kernels; torch supplies device
memory and the current stream.  There is no fallback: if the library is not built, or
there is no GPU, calls raise."""
from __future__ import annotations

import ctypes
import os

from .build import LIB_PATH

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, ENOSYS = 0, -1, -2, -3, -4, -5
BITSLICED, ROWMAJOR_U32, ROWMAJOR_F32 = 0, 1, 2
SCHED_AUTO, SCHED_ONE_WAVE, SCHED_SPLIT, SCHED_SPLIT4 = 0, 1, 2, 3
TRANSPOSE_AUTO, TRANSPOSE_FUSED, TRANSPOSE_STAGED = 0, 1, 2
MAX_BITS_PER_IV = 1 << 40
PACKED_STATE_BYTES = 25

EXPORTED = [
    "mickey_init", "mickey_init_on_stream", "mickey_rekey", "mickey_generate", "mickey_generate_rowmajor",
    "mickey_free", "mickey_set_stream", "mickey_set_word_bits", "mickey_set_schedule", "mickey_set_transpose", "mickey_num_instances",
    "mickey_bits_generated", "mickey_plane_pitch", "mickey_state_export", "mickey_state_import",
    "mickey_sync", "mickey_last_error", "mickey_last_error_message", "mickey_ops_per_clock",
    "mickey_generate_batch", "mickey_instance_bits", "mickey_state_host_bytes", "mickey_state_export_host",
    "mickey_state_import_host", "mickey_debug_fail_launch", "mickey_generate_rowmajor_noalloc",
    "mickey_batch_create", "mickey_batch_set", "mickey_batch_run", "mickey_batch_sync", "mickey_batch_stream",
    "mickey_batch_set_params", "mickey_batch_get_params", "mickey_batch_autotune", "mickey_batch_free",
    "mickey_batch_set_latency_threshold", "mickey_batch_get_routing",
    "mickey_server_create", "mickey_server_submit", "mickey_server_step", "mickey_server_poll",
    "mickey_server_result", "mickey_server_copy", "mickey_server_release", "mickey_server_stats",
    "mickey_server_state", "mickey_server_stream", "mickey_server_free", "mickey_server_submit_many",
    "mickey_server_release_many", "mickey_server_times_many", "mickey_server_wait",
    "mickey_server_latency_words_many",
    "mickey_server_set_chunk", "mickey_server_poll_chunks", "mickey_server_release_chunks",
    "mickey_server_copy_chunk", "mickey_server_set_kernel", "mickey_server_set_latency",
    "grain_init", "grain_rekey", "grain_generate", "grain_generate_rowmajor", "grain_free", "grain_set_stream",
    "grain_num_instances", "grain_bits_generated", "grain_plane_pitch", "grain_state_export",
    "grain_state_import", "grain_sync", "grain_ops_per_clock",
    "aes_ctr_init", "aes_ctr_generate", "aes_ctr_generate_rowmajor", "aes_ctr_seek", "aes_ctr_free",
    "aes_ctr_set_stream", "aes_ctr_num_instances", "aes_ctr_bits_generated", "aes_ctr_plane_pitch",
    "aes_ctr_sync", "aes_ctr_ops_per_block",
    "mickey128_init", "mickey128_generate", "mickey128_sync", "mickey128_export", "mickey128_free",
    "mickey128_num_instances", "mickey128_bits_generated", "mickey128_plane_pitch", "mickey128_ops_per_clock",
]
GRAIN_PACKED_STATE_BYTES = 20

_lib = None


class MickeyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


def load_library():
    """Load lib/libmickey.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmickey.so is not built (run __graft_entry__.build()): " + LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u64, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
    L.mickey_init.argtypes = [vp, vp, vp, sz]
    L.mickey_init.restype = vp
    L.mickey_init_on_stream.argtypes = [vp, vp, vp, sz, vp]
    L.mickey_init_on_stream.restype = vp
    L.mickey_rekey.argtypes = [vp, vp, vp, vp]
    L.mickey_rekey.restype = i
    L.mickey_generate.argtypes = [vp, u64, vp, i]
    L.mickey_generate.restype = i
    L.mickey_generate_rowmajor.argtypes = [vp, u64, vp, vp]
    L.mickey_generate_rowmajor.restype = i
    L.mickey_free.argtypes = [vp]
    L.mickey_free.restype = None
    L.mickey_set_stream.argtypes = [vp, vp]
    L.mickey_set_stream.restype = i
    L.mickey_set_word_bits.argtypes = [vp, i]
    L.mickey_set_word_bits.restype = i
    L.mickey_set_schedule.argtypes = [vp, i]
    L.mickey_set_schedule.restype = i
    L.mickey_set_transpose.argtypes = [vp, i]
    L.mickey_set_transpose.restype = i
    L.mickey_num_instances.argtypes = [vp]
    L.mickey_num_instances.restype = sz
    L.mickey_bits_generated.argtypes = [vp]
    L.mickey_bits_generated.restype = u64
    L.mickey_plane_pitch.argtypes = [sz]
    L.mickey_plane_pitch.restype = sz
    L.mickey_state_export.argtypes = [vp, vp, ctypes.POINTER(u64)]
    L.mickey_state_export.restype = i
    L.mickey_state_import.argtypes = [vp, vp, u64]
    L.mickey_state_import.restype = i
    L.mickey_sync.argtypes = [vp]
    L.mickey_sync.restype = i
    L.mickey_last_error.argtypes = []
    L.mickey_last_error.restype = i
    L.mickey_last_error_message.argtypes = []
    L.mickey_last_error_message.restype = ctypes.c_char_p
    L.mickey_ops_per_clock.argtypes = []
    L.mickey_ops_per_clock.restype = i
    L.mickey_generate_rowmajor_noalloc.argtypes = [vp, u64, vp, vp]
    L.mickey_generate_rowmajor_noalloc.restype = i
    L.mickey_generate_batch.argtypes = [vp, vp, sz]
    L.mickey_generate_batch.restype = i
    L.mickey_instance_bits.argtypes = [vp, sz]
    L.mickey_instance_bits.restype = u64
    L.mickey_state_host_bytes.argtypes = [vp]
    L.mickey_state_host_bytes.restype = sz
    L.mickey_state_export_host.argtypes = [vp, vp, sz]
    L.mickey_state_export_host.restype = i
    L.mickey_state_import_host.argtypes = [vp, vp, sz]
    L.mickey_state_import_host.restype = i
    L.mickey_debug_fail_launch.argtypes = [i]
    L.mickey_debug_fail_launch.restype = i
    L.mickey_batch_create.argtypes = [sz, vp]
    L.mickey_batch_create.restype = vp
    L.mickey_batch_set.argtypes = [vp, vp, vp, vp, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_void_p), sz]
    L.mickey_batch_set.restype = i
    for name in ("mickey_batch_run", "mickey_batch_sync"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = i
    L.mickey_batch_stream.argtypes = [vp]
    L.mickey_batch_stream.restype = vp
    L.mickey_batch_set_params.argtypes = [vp, i, i]
    L.mickey_batch_set_params.restype = i
    L.mickey_batch_get_params.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
    L.mickey_batch_get_params.restype = i
    L.mickey_batch_autotune.argtypes = [vp, u64, ctypes.c_char_p]
    L.mickey_batch_autotune.restype = i
    L.mickey_batch_free.argtypes = [vp]
    L.mickey_batch_free.restype = None
    L.mickey_batch_set_latency_threshold.argtypes = [vp, u64]
    L.mickey_batch_set_latency_threshold.restype = i
    L.mickey_batch_get_routing.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_double)]
    L.mickey_batch_get_routing.restype = i
    L.mickey_server_create.argtypes = [vp, sz, ctypes.c_uint32, u64, vp]
    L.mickey_server_create.restype = vp
    L.mickey_server_submit.argtypes = [vp, ctypes.c_uint32, u64]
    L.mickey_server_submit.restype = ctypes.c_int64
    L.mickey_server_step.argtypes = [vp]
    L.mickey_server_step.restype = i
    L.mickey_server_poll.argtypes = [vp, ctypes.POINTER(u64), sz]
    L.mickey_server_poll.restype = ctypes.c_int64
    L.mickey_server_result.argtypes = [vp, u64, ctypes.POINTER(vp), ctypes.POINTER(u64)]
    L.mickey_server_result.restype = i
    L.mickey_server_copy.argtypes = [vp, u64, vp, u64]
    L.mickey_server_copy.restype = i
    L.mickey_server_release.argtypes = [vp, u64]
    L.mickey_server_release.restype = i
    L.mickey_server_stats.argtypes = [vp, ctypes.POINTER(u64)]
    L.mickey_server_stats.restype = i
    L.mickey_server_state.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(vp), ctypes.POINTER(u64)]
    L.mickey_server_state.restype = i
    L.mickey_server_stream.argtypes = [vp]
    L.mickey_server_stream.restype = vp
    L.mickey_server_free.argtypes = [vp]
    L.mickey_server_free.restype = None
    L.mickey_server_submit_many.argtypes = [vp, vp, vp, sz, vp]
    L.mickey_server_submit_many.restype = i
    L.mickey_server_release_many.argtypes = [vp, vp, sz]
    L.mickey_server_release_many.restype = i
    L.mickey_server_times_many.argtypes = [vp, vp, sz, vp]
    L.mickey_server_times_many.restype = i
    L.mickey_server_latency_words_many.argtypes = [vp, vp, sz, vp]
    L.mickey_server_latency_words_many.restype = i
    L.mickey_server_wait.argtypes = [vp]
    L.mickey_server_wait.restype = i
    L.mickey_server_set_latency.argtypes = [vp, ctypes.c_uint32, u64, u64]
    L.mickey_server_set_latency.restype = i
    L.mickey_server_set_kernel.argtypes = [vp, i, i]
    L.mickey_server_set_kernel.restype = i
    L.mickey_server_set_chunk.argtypes = [vp, u64]
    L.mickey_server_set_chunk.restype = i
    L.mickey_server_poll_chunks.argtypes = [vp, vp, sz]
    L.mickey_server_poll_chunks.restype = ctypes.c_int64
    L.mickey_server_release_chunks.argtypes = [vp, vp, sz]
    L.mickey_server_release_chunks.restype = i
    L.mickey_server_copy_chunk.argtypes = [vp, u64, vp, u64]
    L.mickey_server_copy_chunk.restype = i
    L.grain_init.argtypes = [vp, vp, sz, vp]
    L.grain_init.restype = vp
    L.grain_rekey.argtypes = [vp, vp, vp]
    L.grain_rekey.restype = i
    L.grain_generate.argtypes = [vp, u64, vp, i]
    L.grain_generate.restype = i
    L.grain_generate_rowmajor.argtypes = [vp, u64, vp, vp]
    L.grain_generate_rowmajor.restype = i
    L.grain_free.argtypes = [vp]
    L.grain_free.restype = None
    L.grain_set_stream.argtypes = [vp, vp]
    L.grain_set_stream.restype = i
    L.grain_num_instances.argtypes = [vp]
    L.grain_num_instances.restype = sz
    L.grain_bits_generated.argtypes = [vp]
    L.grain_bits_generated.restype = u64
    L.grain_plane_pitch.argtypes = [sz]
    L.grain_plane_pitch.restype = sz
    L.grain_state_export.argtypes = [vp, vp, ctypes.POINTER(u64)]
    L.grain_state_export.restype = i
    L.grain_state_import.argtypes = [vp, vp, u64]
    L.grain_state_import.restype = i
    L.grain_sync.argtypes = [vp]
    L.grain_sync.restype = i
    L.grain_ops_per_clock.argtypes = []
    L.grain_ops_per_clock.restype = i
    L.aes_ctr_init.argtypes = [vp, vp, sz, vp]
    L.aes_ctr_init.restype = vp
    L.aes_ctr_generate.argtypes = [vp, u64, vp, i]
    L.aes_ctr_generate.restype = i
    L.aes_ctr_generate_rowmajor.argtypes = [vp, u64, vp, vp]
    L.aes_ctr_generate_rowmajor.restype = i
    L.aes_ctr_seek.argtypes = [vp, u64]
    L.aes_ctr_seek.restype = i
    L.aes_ctr_free.argtypes = [vp]
    L.aes_ctr_free.restype = None
    L.aes_ctr_set_stream.argtypes = [vp, vp]
    L.aes_ctr_set_stream.restype = i
    L.aes_ctr_num_instances.argtypes = [vp]
    L.aes_ctr_num_instances.restype = sz
    L.aes_ctr_bits_generated.argtypes = [vp]
    L.aes_ctr_bits_generated.restype = u64
    L.aes_ctr_plane_pitch.argtypes = [sz]
    L.aes_ctr_plane_pitch.restype = sz
    L.aes_ctr_sync.argtypes = [vp]
    L.aes_ctr_sync.restype = i
    L.aes_ctr_ops_per_block.argtypes = []
    L.aes_ctr_ops_per_block.restype = i
    L.mickey128_init.argtypes = [vp, vp, vp, sz, vp]
    L.mickey128_init.restype = vp
    L.mickey128_generate.argtypes = [vp, u64, vp]
    L.mickey128_generate.restype = i
    L.mickey128_sync.argtypes = [vp]
    L.mickey128_sync.restype = i
    L.mickey128_export.argtypes = [vp, vp]
    L.mickey128_export.restype = i
    L.mickey128_free.argtypes = [vp]
    L.mickey128_free.restype = None
    L.mickey128_num_instances.argtypes = [vp]
    L.mickey128_num_instances.restype = sz
    L.mickey128_bits_generated.argtypes = [vp]
    L.mickey128_bits_generated.restype = u64
    L.mickey128_plane_pitch.argtypes = [sz]
    L.mickey128_plane_pitch.restype = sz
    L.mickey128_ops_per_clock.argtypes = []
    L.mickey128_ops_per_clock.restype = i
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != OK:
        L = load_library()
        raise MickeyError(rc, L.mickey_last_error_message().decode())


def plane_pitch(n: int) -> int:
    return int(load_library().mickey_plane_pitch(n))


def ops_per_clock() -> int:
    return int(load_library().mickey_ops_per_clock())


def debug_fail_launch(k: int) -> None:
    """Make the k-th launch from now fail as if the device had refused it (0 cancels)."""
    _check(load_library().mickey_debug_fail_launch(int(k)))


# mickey_req: instance, nbits, out (device address), layout, and the struct's tail padding
REQ_DTYPE = [("instance", "<u8"), ("nbits", "<u8"), ("out", "<u8"), ("layout", "<i4"), ("pad", "<i4")]


def _dev_ptr(t, name: str, nbytes: int):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError("%s holds %d bytes, needs %d" % (name, t.numel() * t.element_size(), nbytes))
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Mickey:
    """n bitsliced MICKEY 2.0 instances resident on the GPU (mickey_state)."""

    def __init__(self, keys, ivs, iv_bits=None, stream=None):
        n = int(keys.shape[0])
        L = load_library()
        kp = _dev_ptr(keys, "keys", 10 * n)
        vp = _dev_ptr(ivs, "ivs", 10 * n)
        bp = None if iv_bits is None else _dev_ptr(iv_bits, "iv_bits", n)
        self._stream = stream
        h = L.mickey_init_on_stream(kp, vp, bp, n, _stream_handle(stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.n = n

    def rekey(self, keys, ivs, iv_bits=None) -> None:
        """Re-initialise all n instances with new keys/IVs (mickey_rekey)."""
        kp = _dev_ptr(keys, "keys", 10 * self.n)
        vp = _dev_ptr(ivs, "ivs", 10 * self.n)
        bp = None if iv_bits is None else _dev_ptr(iv_bits, "iv_bits", self.n)
        _check(load_library().mickey_rekey(self._h, kp, vp, bp))

    # -- properties
    @property
    def bits_generated(self) -> int:
        return int(load_library().mickey_bits_generated(self._h))

    @property
    def pitch(self) -> int:
        return plane_pitch(self.n)

    def set_word_bits(self, bits: int) -> None:
        _check(load_library().mickey_set_word_bits(self._h, int(bits)))

    def set_schedule(self, schedule: int) -> None:
        """SCHED_AUTO, SCHED_ONE_WAVE, SCHED_SPLIT or SCHED_SPLIT4 (mickey_set_schedule)."""
        _check(load_library().mickey_set_schedule(self._h, int(schedule)))

    def set_transpose(self, mode: int) -> None:
        """TRANSPOSE_AUTO, TRANSPOSE_FUSED or TRANSPOSE_STAGED (mickey_set_transpose)."""
        _check(load_library().mickey_set_transpose(self._h, int(mode)))

    def set_stream(self, stream) -> None:
        _check(load_library().mickey_set_stream(self._h, _stream_handle(stream)))
        self._stream = stream

    # -- generation
    def generate(self, nbits: int, layout: int = BITSLICED, out=None):
        import torch
        nbits = int(nbits)
        if layout == BITSLICED:
            nbytes = nbits * self.pitch
            if out is None:
                out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        elif layout in (ROWMAJOR_U32, ROWMAJOR_F32):
            nbytes = self.n * (nbits // 32) * 4  # the library rejects nbits % 32 != 0
            if out is None:
                dt = torch.int32 if layout == ROWMAJOR_U32 else torch.float32
                out = torch.empty((self.n, nbits // 32), dtype=dt, device="cuda")
        else:
            raise ValueError("unknown layout %r" % layout)
        p = _dev_ptr(out, "out", nbytes)
        _check(load_library().mickey_generate(self._h, nbits, p, int(layout)))
        return out

    def generate_rowmajor(self, nbits: int, out_u32=None, out_f32=None, want_u32=True, want_f32=True):
        import torch
        nbits = int(nbits)
        if want_u32 and out_u32 is None:
            out_u32 = torch.empty((self.n, nbits // 32), dtype=torch.int32, device="cuda")
        if want_f32 and out_f32 is None:
            out_f32 = torch.empty((self.n, nbits // 32), dtype=torch.float32, device="cuda")
        nbytes = self.n * (nbits // 32) * 4
        pu = None if out_u32 is None else _dev_ptr(out_u32, "out_u32", nbytes)
        pf = None if out_f32 is None else _dev_ptr(out_f32, "out_f32", nbytes)
        _check(load_library().mickey_generate_rowmajor(self._h, nbits, pu, pf))
        return out_u32, out_f32

    def generate_batch(self, instances, nbits, outs, layouts=ROWMAJOR_U32) -> None:
        """Per-instance requests (mickey_generate_batch): request k resumes instance
        instances[k] for nbits[k] bits into outs[k] (a CUDA tensor of nbits[k]/32 words, or
        a device address), with layouts[k] ROWMAJOR_U32 or ROWMAJOR_F32 (one value for all)."""
        import numpy as np
        n = len(instances)
        req = np.zeros(n, dtype=REQ_DTYPE)
        req["instance"] = np.asarray(instances, dtype=np.uint64)
        req["nbits"] = np.asarray(nbits, dtype=np.uint64)
        req["layout"] = np.broadcast_to(np.asarray(layouts, dtype=np.int32), (n,))
        ptrs = []
        for k, o in enumerate(outs):
            if isinstance(o, int):
                ptrs.append(o)
            else:
                ptrs.append(_dev_ptr(o, "outs[%d]" % k, int(req["nbits"][k]) // 8).value or 0)
        req["out"] = np.asarray(ptrs, dtype=np.uint64)
        _check(load_library().mickey_generate_batch(self._h, req.ctypes.data, n))

    def instance_bits(self, i: int) -> int:
        v = int(load_library().mickey_instance_bits(self._h, int(i)))
        if v == (1 << 64) - 1:
            _check(load_library().mickey_last_error())
        return v

    # -- state
    def export_host(self) -> bytes:
        """The state in host form (mickey_state_export_host): header, packed registers,
        per-instance bit counters."""
        import numpy as np
        L = load_library()
        buf = np.zeros(int(L.mickey_state_host_bytes(self._h)), dtype=np.uint8)
        _check(L.mickey_state_export_host(self._h, buf.ctypes.data, buf.nbytes))
        return buf.tobytes()

    def import_host(self, blob: bytes) -> None:
        import numpy as np
        a = np.frombuffer(bytes(blob), dtype=np.uint8)
        _check(load_library().mickey_state_import_host(self._h, a.ctypes.data, a.nbytes))

    def export_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.n, PACKED_STATE_BYTES), dtype=torch.uint8, device="cuda")
        bits = ctypes.c_uint64(0)
        _check(load_library().mickey_state_export(self._h, _dev_ptr(out, "packed", 25 * self.n),
                                                  ctypes.byref(bits)))
        return out, int(bits.value)

    def import_state(self, packed, bits_generated: int) -> None:
        _check(load_library().mickey_state_import(self._h, _dev_ptr(packed, "packed", 25 * self.n),
                                                  int(bits_generated)))

    def sync(self) -> None:
        _check(load_library().mickey_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().mickey_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """mickey_batch: many fresh requests in one persistent, graph-captured launch."""

    def __init__(self, max_requests: int, stream=None):
        L = load_library()
        h = L.mickey_batch_create(int(max_requests), None if stream is None else ctypes.c_void_p(stream.cuda_stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.max_requests = int(max_requests)
        self._keep = None

    @property
    def stream_handle(self) -> int:
        return int(load_library().mickey_batch_stream(self._h) or 0)

    def set(self, keys, ivs, iv_bits, nbits, out_ptrs) -> None:
        """keys/ivs uint8 [nreq,10] and iv_bits uint8 [nreq] (or None) CUDA tensors;
        nbits: host sequence of lengths (multiples of 32); out_ptrs: host sequence of
        device addresses (int) receiving nbits/32 row-major words each."""
        import numpy as np
        n = int(keys.shape[0])
        nb = np.ascontiguousarray(np.asarray(nbits, dtype=np.uint64))
        op = np.ascontiguousarray(np.asarray(out_ptrs, dtype=np.uint64))
        assert nb.shape == (n,) and op.shape == (n,)
        kp = _dev_ptr(keys, "keys", 10 * n)
        vp = _dev_ptr(ivs, "ivs", 10 * n)
        bp = None if iv_bits is None else _dev_ptr(iv_bits, "iv_bits", n)
        self._keep = (keys, ivs, iv_bits)  # device inputs must outlive the runs
        _check(load_library().mickey_batch_set(
            self._h, kp, vp, bp, nb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            op.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)), n))

    def run(self) -> None:
        _check(load_library().mickey_batch_run(self._h))

    def sync(self) -> None:
        _check(load_library().mickey_batch_sync(self._h))

    def set_params(self, unroll: int = 0, waves_per_block: int = 0) -> None:
        _check(load_library().mickey_batch_set_params(self._h, int(unroll), int(waves_per_block)))

    def get_params(self):
        u, w = ctypes.c_int(0), ctypes.c_int(0)
        _check(load_library().mickey_batch_get_params(self._h, ctypes.byref(u), ctypes.byref(w)))
        return u.value, w.value

    LATENCY_OFF = (1 << 64) - 1

    def set_latency_threshold(self, bits: int) -> None:
        """0: automatic size-aware routing; LATENCY_OFF: all bitsliced; else a threshold."""
        _check(load_library().mickey_batch_set_latency_threshold(self._h, int(bits)))

    def routing(self):
        """(threshold in bits or None, requests in latency mode, latency/bitsliced clock ratio)"""
        t, n, r = ctypes.c_uint64(0), ctypes.c_size_t(0), ctypes.c_double(0)
        _check(load_library().mickey_batch_get_routing(self._h, ctypes.byref(t), ctypes.byref(n), ctypes.byref(r)))
        return (None if t.value == self.LATENCY_OFF else int(t.value)), int(n.value), float(r.value)

    def autotune(self, cap_bits: int, cache_path=None):
        _check(load_library().mickey_batch_autotune(
            self._h, int(cap_bits), None if cache_path is None else str(cache_path).encode()))
        return self.get_params()

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().mickey_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """mickey_server: resident states, resumable requests, continuous batching."""

    STAT_KEYS = ("waiting", "running", "admitted", "finished", "steps", "quantum_ns", "bits_delivered",
                 "free_budget_words", "host_wait_ns", "host_retire_ns", "host_admit_ns", "gpu_ns")

    def __init__(self, init: "Mickey", nslices: int, quantum_clocks: int, budget_bytes: int, stream=None):
        L = load_library()
        h = L.mickey_server_create(init._h, int(nslices), int(quantum_clocks), int(budget_bytes),
                                   None if stream is None else ctypes.c_void_p(stream.cuda_stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.n = init.n
        self.quantum_clocks = int(quantum_clocks)

    def set_latency(self, streams: int, threshold_bits: int = 1 << 20, clocks_per_quantum: int = 0) -> None:
        """Latency-stream routing (mickey_server_set_latency); clocks_per_quantum 0 means 8
        quanta's worth of clocks of the server's quantum."""
        cpq = int(clocks_per_quantum) or 8 * self.quantum_clocks
        _check(load_library().mickey_server_set_latency(self._h, int(streams), int(threshold_bits), cpq))

    def set_kernel(self, schedule: int = SCHED_AUTO, transpose: int = TRANSPOSE_AUTO) -> None:
        """Kernels of the following quanta (mickey_server_set_kernel)."""
        _check(load_library().mickey_server_set_kernel(self._h, int(schedule), int(transpose)))

    def submit(self, state_id: int, nbits: int) -> int:
        r = load_library().mickey_server_submit(self._h, int(state_id), int(nbits))
        if r < 0:
            _check(int(r))
        return int(r)

    def submit_many(self, sids, nbits):
        import numpy as np
        s = np.ascontiguousarray(sids, dtype=np.uint32)
        b = np.ascontiguousarray(nbits, dtype=np.uint64)
        ids = np.zeros(len(s), dtype=np.int64)
        _check(load_library().mickey_server_submit_many(self._h, s.ctypes.data, b.ctypes.data, len(s),
                                                        ids.ctypes.data))
        return ids

    def release_many(self, ids) -> None:
        import numpy as np
        a = np.ascontiguousarray(ids, dtype=np.uint64)
        _check(load_library().mickey_server_release_many(self._h, a.ctypes.data, len(a)))

    def times_many(self, ids):
        import numpy as np
        a = np.ascontiguousarray(ids, dtype=np.uint64)
        out = np.zeros((len(a), 3), dtype=np.uint64)
        _check(load_library().mickey_server_times_many(self._h, a.ctypes.data, len(a), out.ctypes.data))
        return out

    def latency_words_many(self, ids):
        """Words of each request admitted to latency streams so far."""
        import numpy as np
        a = np.ascontiguousarray(ids, dtype=np.uint64)
        out = np.zeros(len(a), dtype=np.uint64)
        _check(load_library().mickey_server_latency_words_many(self._h, a.ctypes.data, len(a), out.ctypes.data))
        return out

    def step(self) -> None:
        _check(load_library().mickey_server_step(self._h))

    def wait(self) -> None:
        _check(load_library().mickey_server_wait(self._h))

    def poll(self, cap: int = 1 << 20):
        """Ids of completed requests since the last poll (numpy uint64 array)."""
        import numpy as np
        buf = np.empty(cap, dtype=np.uint64)
        k = load_library().mickey_server_poll(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cap)
        if k < 0:
            _check(int(k))
        return buf[:k].copy()

    def times(self, rid: int):
        """(arrival, admission, completion) in ns of the steady clock; raises MickeyError
        with code ERANGE for a request refused at the 2^40-bit limit."""
        t = (ctypes.c_uint64 * 3)()
        _check(load_library().mickey_server_result(self._h, int(rid), None, t))
        return int(t[0]), int(t[1]), int(t[2])

    # -- chunked delivery
    CHUNK_DTYPE = [("request", "<u8"), ("handle", "<u8"), ("offset", "<u8"), ("words", "<u8"), ("out", "<u8"),
                   ("last", "<u8")]

    def set_chunk(self, chunk_bytes: int) -> None:
        """Deliver later submissions in chunks of chunk_bytes (0: whole requests)."""
        _check(load_library().mickey_server_set_chunk(self._h, int(chunk_bytes)))

    def poll_chunks(self, cap: int = 1 << 20):
        """Chunks finished since the last call: numpy structured array with fields
        request, handle, offset (first word in the request's stream), words, out (device
        address) and last."""
        import numpy as np
        buf = np.empty(cap, dtype=self.CHUNK_DTYPE)
        k = load_library().mickey_server_poll_chunks(self._h, buf.ctypes.data, cap)
        if k < 0:
            _check(int(k))
        return buf[:k].copy()

    def release_chunks(self, handles) -> None:
        import numpy as np
        a = np.ascontiguousarray(handles, dtype=np.uint64)
        _check(load_library().mickey_server_release_chunks(self._h, a.ctypes.data, len(a)))

    def copy_chunk(self, handle: int, dst, nwords: int) -> None:
        _check(load_library().mickey_server_copy_chunk(self._h, int(handle), _dev_ptr(dst, "dst", 4 * nwords),
                                                       int(nwords)))

    def copy(self, rid: int, dst, nwords: int) -> None:
        _check(load_library().mickey_server_copy(self._h, int(rid), _dev_ptr(dst, "dst", 4 * nwords), int(nwords)))

    def release(self, rid: int) -> None:
        _check(load_library().mickey_server_release(self._h, int(rid)))

    def stats(self) -> dict:
        out = (ctypes.c_uint64 * len(self.STAT_KEYS))()
        _check(load_library().mickey_server_stats(self._h, out))
        return dict(zip(self.STAT_KEYS, [int(v) for v in out]))

    def state_bits(self, sid: int) -> int:
        b = ctypes.c_uint64()
        _check(load_library().mickey_server_state(self._h, int(sid), None, ctypes.byref(b)))
        return int(b.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().mickey_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grain_ops_per_clock() -> int:
    return int(load_library().grain_ops_per_clock())


class Grain:
    """n bitsliced Grain (v1) instances resident on the GPU (grain_state): 80-bit keys
    (n x 10 bytes) and 64-bit IVs (n x 8 bytes), bits least significant first."""

    def __init__(self, keys, ivs, stream=None):
        n = int(keys.shape[0])
        L = load_library()
        h = L.grain_init(_dev_ptr(keys, "keys", 10 * n), _dev_ptr(ivs, "ivs", 8 * n), n, _stream_handle(stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.n = n

    def rekey(self, keys, ivs) -> None:
        _check(load_library().grain_rekey(self._h, _dev_ptr(keys, "keys", 10 * self.n),
                                          _dev_ptr(ivs, "ivs", 8 * self.n)))

    @property
    def bits_generated(self) -> int:
        return int(load_library().grain_bits_generated(self._h))

    @property
    def pitch(self) -> int:
        return int(load_library().grain_plane_pitch(self.n))

    def set_stream(self, stream) -> None:
        _check(load_library().grain_set_stream(self._h, _stream_handle(stream)))

    def generate(self, nbits: int, layout: int = BITSLICED, out=None):
        import torch
        nbits = int(nbits)
        if layout == BITSLICED:
            nbytes = nbits * self.pitch
            if out is None:
                out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        elif layout in (ROWMAJOR_U32, ROWMAJOR_F32):
            nbytes = self.n * (nbits // 32) * 4
            if out is None:
                dt = torch.int32 if layout == ROWMAJOR_U32 else torch.float32
                out = torch.empty((self.n, nbits // 32), dtype=dt, device="cuda")
        else:
            raise ValueError("unknown layout %r" % layout)
        _check(load_library().grain_generate(self._h, nbits, _dev_ptr(out, "out", nbytes), int(layout)))
        return out

    def generate_rowmajor(self, nbits: int, out_u32=None, out_f32=None, want_u32=True, want_f32=True):
        import torch
        nbits = int(nbits)
        if want_u32 and out_u32 is None:
            out_u32 = torch.empty((self.n, nbits // 32), dtype=torch.int32, device="cuda")
        if want_f32 and out_f32 is None:
            out_f32 = torch.empty((self.n, nbits // 32), dtype=torch.float32, device="cuda")
        nbytes = self.n * (nbits // 32) * 4
        pu = None if out_u32 is None else _dev_ptr(out_u32, "out_u32", nbytes)
        pf = None if out_f32 is None else _dev_ptr(out_f32, "out_f32", nbytes)
        _check(load_library().grain_generate_rowmajor(self._h, nbits, pu, pf))
        return out_u32, out_f32

    def export_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.n, GRAIN_PACKED_STATE_BYTES), dtype=torch.uint8, device="cuda")
        bits = ctypes.c_uint64(0)
        _check(load_library().grain_state_export(self._h, _dev_ptr(out, "packed", 20 * self.n), ctypes.byref(bits)))
        return out, int(bits.value)

    def import_state(self, packed, bits_generated: int) -> None:
        _check(load_library().grain_state_import(self._h, _dev_ptr(packed, "packed", 20 * self.n),
                                                 int(bits_generated)))

    def sync(self) -> None:
        _check(load_library().grain_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().grain_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def aes_ops_per_block() -> int:
    return int(load_library().aes_ctr_ops_per_block())


class AesCtr:
    """n AES-128 counter-mode streams under one key (aes_ctr_state): stream i's block j is
    AES_K(nonce_i || j as 64-bit big-endian).  key: 16 bytes, nonces: n x 8 bytes (device)."""

    def __init__(self, key, nonces, stream=None):
        n = int(nonces.shape[0])
        L = load_library()
        h = L.aes_ctr_init(_dev_ptr(key, "key", 16), _dev_ptr(nonces, "nonces", 8 * n), n, _stream_handle(stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.n = n

    @property
    def bits_generated(self) -> int:
        return int(load_library().aes_ctr_bits_generated(self._h))

    @property
    def pitch(self) -> int:
        return int(load_library().aes_ctr_plane_pitch(self.n))

    def seek(self, block: int) -> None:
        _check(load_library().aes_ctr_seek(self._h, int(block)))

    def set_stream(self, stream) -> None:
        _check(load_library().aes_ctr_set_stream(self._h, _stream_handle(stream)))

    def generate(self, nbits: int, layout: int = BITSLICED, out=None):
        import torch
        nbits = int(nbits)
        if layout == BITSLICED:
            nbytes = nbits * self.pitch
            if out is None:
                out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        elif layout in (ROWMAJOR_U32, ROWMAJOR_F32):
            nbytes = self.n * (nbits // 32) * 4
            if out is None:
                dt = torch.int32 if layout == ROWMAJOR_U32 else torch.float32
                out = torch.empty((self.n, nbits // 32), dtype=dt, device="cuda")
        else:
            raise ValueError("unknown layout %r" % layout)
        _check(load_library().aes_ctr_generate(self._h, nbits, _dev_ptr(out, "out", nbytes), int(layout)))
        return out

    def generate_rowmajor(self, nbits: int, out_u32=None, out_f32=None, want_u32=True, want_f32=True):
        import torch
        nbits = int(nbits)
        if want_u32 and out_u32 is None:
            out_u32 = torch.empty((self.n, nbits // 32), dtype=torch.int32, device="cuda")
        if want_f32 and out_f32 is None:
            out_f32 = torch.empty((self.n, nbits // 32), dtype=torch.float32, device="cuda")
        nbytes = self.n * (nbits // 32) * 4
        pu = None if out_u32 is None else _dev_ptr(out_u32, "out_u32", nbytes)
        pf = None if out_f32 is None else _dev_ptr(out_f32, "out_f32", nbytes)
        _check(load_library().aes_ctr_generate_rowmajor(self._h, nbits, pu, pf))
        return out_u32, out_f32

    def sync(self) -> None:
        _check(load_library().aes_ctr_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().aes_ctr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mickey128_ops_per_clock() -> int:
    return int(load_library().mickey128_ops_per_clock())


class Mickey128:
    """n bitsliced MICKEY-128 2.0 instances resident on the GPU (mickey128_state): 128-bit
    keys and IVs (n x 16 bytes, bits MSB first) and IV lengths 0..128 (n bytes, or None
    for 128), all device tensors.  Output: bit-planes of pitch n_pad/8 bytes."""

    def __init__(self, keys, ivs, iv_bits=None, stream=None):
        n = int(keys.shape[0])
        L = load_library()
        pb = None if iv_bits is None else _dev_ptr(iv_bits, "iv_bits", n)
        h = L.mickey128_init(_dev_ptr(keys, "keys", 16 * n), _dev_ptr(ivs, "ivs", 16 * n), pb, n,
                             _stream_handle(stream))
        if not h:
            raise MickeyError(L.mickey_last_error(), L.mickey_last_error_message().decode())
        self._h = ctypes.c_void_p(h)
        self.n = n

    @property
    def bits_generated(self) -> int:
        return int(load_library().mickey128_bits_generated(self._h))

    @property
    def pitch(self) -> int:
        return int(load_library().mickey128_plane_pitch(self.n))

    def generate(self, nbits: int, out=None):
        import torch
        nbits = int(nbits)
        nbytes = nbits * self.pitch
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(load_library().mickey128_generate(self._h, nbits, _dev_ptr(out, "out", nbytes)))
        return out

    def export_planes(self, out=None):
        """The 320 register planes (r_0..r_159, s_0..s_159), pitch bytes each."""
        import torch
        nbytes = 320 * self.pitch
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(load_library().mickey128_export(self._h, _dev_ptr(out, "planes", nbytes)))
        return out

    def sync(self) -> None:
        _check(load_library().mickey128_sync(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().mickey128_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
