"""Python binding of libmickpt.so (include/mickpt.h), argument marshalling only.

Every computation happens in the library's HIP kernels and host runtime; this
module converts torch tensors and Python values to the C structures and back.
It raises ImportError-like RuntimeError when the library is not built: there
is no fallback.

Functions carry the C names:
    ckpt_ctx_create(device, staging_budget) -> ctx
    ckpt_dump(ctx, table, prev=None, opts=None, stream=None) -> (rc, Image|None, result)
    ckpt_restore(ctx, image, table, opts=None, stream=None) -> (rc, result)
    ckpt_merge(base, delta) -> (rc, Image|None)
    ckpt_image_import(data) -> (rc, Image|None)
A table is a list of (id, tensor) pairs (any dtype; the tensor's bytes are
the allocation) or of (id, device_pointer, size) triples.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmickpt.so")

CKPT_OK = 0
CKPT_EINVAL = -1
CKPT_ENOMEM = -2
CKPT_EHIP = -3
CKPT_ECORRUPT = -4
CKPT_EMISMATCH = -5
CKPT_EBASE = -6
CKPT_ETIMEOUT = -7
CKPT_EIO = -8
CKPT_ELIMIT = -9
KIND_ZERO, KIND_DATA, KIND_UNCHANGED, KIND_PACKED = 0, 1, 2, 3
OPT_PER_ALLOC = 1
OPT_GRAPH = 2
OPT_NO_TIMING = 4
OPT_CODEC = 8
NO_CHUNK = (1 << 64) - 1

_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32


class ckpt_alloc(ctypes.Structure):
    _fields_ = [("id", _u64), ("dev_ptr", ctypes.c_void_p), ("size", _u64)]


class ckpt_alloc_table(ctypes.Structure):
    _fields_ = [("v", ctypes.POINTER(ckpt_alloc)), ("n", _u32)]


class ckpt_opts(ctypes.Structure):
    _fields_ = [("chunk_size", _u32), ("wg_threads", _u32), ("copy_streams", _u32), ("slots", _u32),
                ("window_bytes", _u64), ("flags", _u32), ("strict_verify", _u32)]


class ckpt_result(ctypes.Structure):
    _fields_ = [("first_bad_chunk", _u64), ("hip_error", ctypes.c_int32), ("windows", _u32),
                ("n_logical", _u64), ("n_payload", _u64), ("n_chunks", _u64),
                ("n_zero", _u64), ("n_data", _u64), ("n_unchanged", _u64),
                ("link_bytes", _u64), ("ns_total", _u64), ("ns_kernel", _u64), ("ns_link", _u64),
                ("n_packed", _u64), ("reserved", _u64 * 3), ("ns_stage", _u64 * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("reserved", "ns_stage")}
        d["ns_stage"] = list(self.ns_stage)
        return d


class ckpt_request(ctypes.Structure):
    _fields_ = [("kind", _u32), ("tenant", _u32), ("table", ctypes.POINTER(ckpt_alloc_table)),
                ("prev", ctypes.c_void_p), ("img", ctypes.c_void_p), ("deadline_ns", _u64)]


class ckpt_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("failed", _u64), ("bytes_logical", _u64),
                ("bytes_link", _u64), ("launches", _u64), ("max_batch", _u64), ("p50_ns", _u64),
                ("p99_ns", _u64), ("mean_wait_ns", _u64), ("max_wait_ns", _u64), ("host_copies", _u64),
                ("host_copy_bytes", _u64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


REQ_DUMP = 1
REQ_RESTORE = 2
_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmickpt.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.ckpt_ctx_create.argtypes = [ctypes.c_int, _u64, ctypes.POINTER(vp)]
        L.ckpt_ctx_create.restype = ctypes.c_int
        L.ckpt_ctx_destroy.argtypes = [vp]
        L.ckpt_ctx_destroy.restype = None
        L.ckpt_dump.argtypes = [vp, ctypes.POINTER(ckpt_alloc_table), vp, ctypes.POINTER(vp),
                                ctypes.POINTER(ckpt_opts), vp, ctypes.POINTER(ckpt_result)]
        L.ckpt_dump.restype = ctypes.c_int
        L.ckpt_dump_into.argtypes = [vp, ctypes.POINTER(ckpt_alloc_table), vp, vp, _u64, ctypes.POINTER(_u64),
                                     ctypes.POINTER(ckpt_opts), vp, ctypes.POINTER(ckpt_result)]
        L.ckpt_dump_into.restype = ctypes.c_int
        L.ckpt_restore.argtypes = [vp, vp, ctypes.POINTER(ckpt_alloc_table), ctypes.POINTER(ckpt_opts), vp,
                                   ctypes.POINTER(ckpt_result)]
        L.ckpt_restore.restype = ctypes.c_int
        L.ckpt_restore_some.argtypes = [vp, vp, ctypes.POINTER(ckpt_alloc_table), ctypes.POINTER(ckpt_opts), vp,
                                   ctypes.POINTER(ckpt_result)]
        L.ckpt_restore_some.restype = ctypes.c_int
        L.ckpt_image_save.argtypes = [vp, ctypes.c_char_p, _u32]
        L.ckpt_image_save.restype = ctypes.c_int
        L.ckpt_image_load.argtypes = [ctypes.c_char_p, _u32, ctypes.POINTER(vp)]
        L.ckpt_image_load.restype = ctypes.c_int
        L.ckpt_dump_file.argtypes = [vp, ctypes.POINTER(ckpt_alloc_table), vp, ctypes.c_char_p, _u32,
                                     ctypes.POINTER(ckpt_opts), vp, ctypes.POINTER(ckpt_result), ctypes.POINTER(vp)]
        L.ckpt_dump_file.restype = ctypes.c_int
        L.ckpt_restore_file.argtypes = [vp, ctypes.c_char_p, _u32, ctypes.POINTER(ckpt_alloc_table),
                                        ctypes.POINTER(ckpt_opts), vp, ctypes.POINTER(ckpt_result)]
        L.ckpt_restore_file.restype = ctypes.c_int
        L.ckpt_merge.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.ckpt_merge.restype = ctypes.c_int
        L.ckpt_image_bytes.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(_u64)]
        L.ckpt_image_bytes.restype = ctypes.c_int
        L.ckpt_image_import.argtypes = [vp, _u64, ctypes.POINTER(vp)]
        L.ckpt_image_import.restype = ctypes.c_int
        L.ckpt_image_free.argtypes = [vp]
        L.ckpt_image_free.restype = None
        L.ckpt_strerror.argtypes = [ctypes.c_int]
        L.ckpt_strerror.restype = ctypes.c_char_p
        L.ckpt_autotune.argtypes = [vp, ctypes.POINTER(ckpt_alloc_table), _u64, _u32, ctypes.POINTER(ckpt_opts),
                                    ctypes.POINTER(ctypes.c_double)]
        L.ckpt_autotune.restype = ctypes.c_int
        L.ckpt_serve_create.argtypes = [vp, _u32, _u64, ctypes.POINTER(vp)]
        L.ckpt_serve_create.restype = ctypes.c_int
        L.ckpt_serve_submit.argtypes = [vp, ctypes.POINTER(ckpt_request), ctypes.POINTER(_u64)]
        L.ckpt_serve_submit.restype = ctypes.c_int
        L.ckpt_serve_poll.argtypes = [vp, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp),
                                      ctypes.POINTER(_u64)]
        L.ckpt_serve_poll.restype = ctypes.c_int
        L.ckpt_serve_drain.argtypes = [vp]
        L.ckpt_serve_drain.restype = ctypes.c_int
        L.ckpt_serve_stats.argtypes = [vp, ctypes.POINTER(ckpt_server_stats)]
        L.ckpt_serve_stats.restype = ctypes.c_int
        L.ckpt_serve_destroy.argtypes = [vp]
        L.ckpt_serve_destroy.restype = None
        L.ckpt_crc32c.argtypes = [vp, _u64]
        L.ckpt_crc32c.restype = _u32
        _lib = L
    return _lib


class _Bytes:
    """Array-interface holder for image bytes; keeps the Image alive while a
    numpy view of it exists."""

    def __init__(self, owner, addr, n):
        self._owner = owner
        self.__array_interface__ = {"shape": (n,), "typestr": "|u1", "data": (addr, False), "version": 3}


class Image:
    """An image owned by the library (pinned host memory); released by free()
    or when the last reference (including numpy views) goes away."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def nbytes(self):
        p, n = ctypes.c_void_p(), _u64()
        lib().ckpt_image_bytes(self.handle, ctypes.byref(p), ctypes.byref(n))
        return n.value

    def view(self):
        """Zero-copy numpy uint8 view of the image bytes (valid until free)."""
        import numpy as np
        p, n = ctypes.c_void_p(), _u64()
        rc = lib().ckpt_image_bytes(self.handle, ctypes.byref(p), ctypes.byref(n))
        if rc != 0:
            raise RuntimeError(ckpt_strerror(rc))
        if n.value == 0:
            return np.zeros(0, np.uint8)
        return np.asarray(_Bytes(self, p.value, n.value))

    def tobytes(self):
        return self.view().tobytes()

    def free(self):
        if self.handle is not None and self.handle.value:
            lib().ckpt_image_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _table(entries):
    n = len(entries)
    arr = (ckpt_alloc * max(n, 1))()
    keep = []
    for i, e in enumerate(entries):
        if len(e) == 2:
            aid, t = e
            keep.append(t)
            arr[i].id = int(aid)
            arr[i].dev_ptr = t.data_ptr() if t.numel() else None
            arr[i].size = t.numel() * t.element_size()
        else:
            aid, ptr, size = e
            arr[i].id = int(aid)
            arr[i].dev_ptr = int(ptr) if ptr else None
            arr[i].size = int(size)
    tab = ckpt_alloc_table(ctypes.cast(arr, ctypes.POINTER(ckpt_alloc)), n)
    return tab, (arr, keep)


def make_opts(chunk_size=0, wg_threads=0, copy_streams=0, slots=0, window_bytes=0, flags=0, strict_verify=0):
    return ckpt_opts(chunk_size, wg_threads, copy_streams, slots, window_bytes, flags, int(strict_verify))


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def ckpt_strerror(rc):
    return lib().ckpt_strerror(rc).decode()


def ckpt_crc32c(data):
    b = bytes(data)
    buf = ctypes.create_string_buffer(b, len(b))
    return int(lib().ckpt_crc32c(buf, len(b)))


def ckpt_ctx_create(device=0, staging_budget=0):
    ctx = ctypes.c_void_p()
    rc = lib().ckpt_ctx_create(int(device), int(staging_budget), ctypes.byref(ctx))
    if rc != 0:
        raise RuntimeError("ckpt_ctx_create: %s" % ckpt_strerror(rc))
    return ctx


def ckpt_ctx_destroy(ctx):
    lib().ckpt_ctx_destroy(ctx)


def ckpt_dump(ctx, table, prev=None, opts=None, stream=None):
    tab, keep = _table(table)
    out = ctypes.c_void_p()
    res = ckpt_result()
    rc = lib().ckpt_dump(ctx, ctypes.byref(tab), prev.handle if prev is not None else None,
                         ctypes.byref(out), ctypes.byref(opts) if opts is not None else None,
                         _stream(stream), ctypes.byref(res))
    return rc, (Image(out.value) if rc == 0 else None), res


def ckpt_dump_into(ctx, table, out, prev=None, opts=None, stream=None):
    """Dump into the caller's host buffer `out` (a writable uint8 numpy
    array); nothing is allocated. Returns (rc, image length, result)."""
    tab, keep = _table(table)
    n = _u64()
    res = ckpt_result()
    rc = lib().ckpt_dump_into(ctx, ctypes.byref(tab), prev.handle if prev is not None else None,
                              ctypes.c_void_p(out.ctypes.data), int(out.nbytes), ctypes.byref(n),
                              ctypes.byref(opts) if opts is not None else None, _stream(stream), ctypes.byref(res))
    return rc, n.value, res


def ckpt_restore(ctx, image, table, opts=None, stream=None):
    tab, keep = _table(table)
    res = ckpt_result()
    rc = lib().ckpt_restore(ctx, image.handle, ctypes.byref(tab),
                            ctypes.byref(opts) if opts is not None else None, _stream(stream), ctypes.byref(res))
    return rc, res


def ckpt_restore_some(ctx, image, table, opts=None, stream=None):
    """On-demand restore of the listed allocations only (matched by id)."""
    tab, keep = _table(table)
    res = ckpt_result()
    rc = lib().ckpt_restore_some(ctx, image.handle, ctypes.byref(tab),
                                 ctypes.byref(opts) if opts is not None else None, _stream(stream), ctypes.byref(res))
    return rc, res


def ckpt_autotune(ctx, table, sample_bytes=0, flags=0):
    tab, keep = _table(table)
    best = ckpt_opts()
    gbps = ctypes.c_double(0)
    rc = lib().ckpt_autotune(ctx, ctypes.byref(tab), int(sample_bytes), int(flags), ctypes.byref(best),
                             ctypes.byref(gbps))
    return rc, best, gbps.value


def ckpt_image_save(image, path, threads=0):
    """Write the image to a file (synced)."""
    return lib().ckpt_image_save(image.handle, os.fsencode(path), int(threads))


def ckpt_image_load(path, threads=0):
    """Read and validate an image file: (rc, Image or None)."""
    out = ctypes.c_void_p()
    rc = lib().ckpt_image_load(os.fsencode(path), int(threads), ctypes.byref(out))
    return rc, (Image(out.value) if rc == 0 else None)


def ckpt_dump_file(ctx, table, path, prev=None, opts=None, stream=None, io_threads=0, keep_image=False):
    """Dump with the image written to `path` while it is copied out:
    (rc, Image or None, result); the image is returned only with keep_image."""
    tab, keep = _table(table)
    out = ctypes.c_void_p()
    res = ckpt_result()
    rc = lib().ckpt_dump_file(ctx, ctypes.byref(tab), prev.handle if prev is not None else None, os.fsencode(path),
                              int(io_threads), ctypes.byref(opts) if opts is not None else None, _stream(stream),
                              ctypes.byref(res), ctypes.byref(out) if keep_image else None)
    return rc, (Image(out.value) if rc == 0 and keep_image else None), res


def ckpt_restore_file(ctx, path, table, opts=None, stream=None, io_threads=0):
    """Restore the image in `path`, uploading windows as the file loads: (rc, result)."""
    tab, keep = _table(table)
    res = ckpt_result()
    rc = lib().ckpt_restore_file(ctx, os.fsencode(path), int(io_threads), ctypes.byref(tab),
                                 ctypes.byref(opts) if opts is not None else None, _stream(stream), ctypes.byref(res))
    return rc, res


def ckpt_merge(base, delta):
    out = ctypes.c_void_p()
    rc = lib().ckpt_merge(base.handle, delta.handle, ctypes.byref(out))
    return rc, (Image(out.value) if rc == 0 else None)


def ckpt_image_import(data):
    import numpy as np
    a = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else data)
    out = ctypes.c_void_p()
    rc = lib().ckpt_image_import(a.ctypes.data if a.size else None, a.size, ctypes.byref(out))
    return rc, (Image(out.value) if rc == 0 else None)


class _Pending:
    """A submitted request's marshalled arguments, kept alive until it is polled."""

    def __init__(self, tab, keep, req):
        self.tab, self.keep, self.req = tab, keep, req


_inflight = {}


def ckpt_serve_create(ctx, max_active=0, budget=0):
    srv = ctypes.c_void_p()
    rc = lib().ckpt_serve_create(ctx, int(max_active), int(budget), ctypes.byref(srv))
    if rc != 0:
        raise RuntimeError("ckpt_serve_create: %s" % ckpt_strerror(rc))
    return srv


def ckpt_serve_submit(srv, kind, table, prev=None, img=None, tenant=0, deadline_ns=0):
    tab, keep = _table(table)
    req = ckpt_request(kind, tenant, ctypes.pointer(tab), prev.handle if prev is not None else None,
                       img.handle if img is not None else None, deadline_ns)
    ticket = _u64()
    rc = lib().ckpt_serve_submit(srv, ctypes.byref(req), ctypes.byref(ticket))
    if rc == 0:
        _inflight[(srv.value, ticket.value)] = _Pending(tab, keep, req)
    return rc, ticket.value


def ckpt_serve_poll(srv, ticket):
    """Returns (done, rc, Image|None, latency_ns)."""
    rc = ctypes.c_int(0)
    out = ctypes.c_void_p()
    lat = _u64()
    done = lib().ckpt_serve_poll(srv, ticket, ctypes.byref(rc), ctypes.byref(out), ctypes.byref(lat))
    if done == 1:
        _inflight.pop((srv.value, ticket), None)
        return True, rc.value, (Image(out.value) if out.value else None), lat.value
    if done < 0:
        raise RuntimeError("ckpt_serve_poll: %s" % ckpt_strerror(done))
    return False, None, None, None


def ckpt_serve_drain(srv):
    return lib().ckpt_serve_drain(srv)


def ckpt_serve_stats(srv):
    st = ckpt_server_stats()
    lib().ckpt_serve_stats(srv, ctypes.byref(st))
    return st


def ckpt_serve_destroy(srv):
    lib().ckpt_serve_destroy(srv)
    for k in [k for k in _inflight if k[0] == srv.value]:
        _inflight.pop(k)
