"""Exact bivariate resultants and integer gcds on the MI355X.

Thin ctypes binding over libsnc.so (C ABI in include/snc.h).  Python only
marshals integers to and from 32-bit two's-complement limbs and provides
device workspaces from PyTorch; every step of the computation runs in the
library's HIP kernels.  If the library is missing the binding raises; there
is no fallback path.

    import paper_1103_4697_amd as snc
    R = snc.resultant_y(f, g)        # f, g: [i][k] integer arrays, y^i x^k
    G = snc.gcd_z(a, b)              # a, b: ascending integer lists
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnc.so")

SNC_OK, SNC_EINVAL, SNC_ERANGE, SNC_ENOMEM, SNC_EDEVICE, SNC_EAGAIN, SNC_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
SNC_ENOTSUP = -7


class SncError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"snc status {status} ({_status_name(status)}): {msg}")
        self.status = status


class Bipoly(C.Structure):
    _fields_ = [("limbs", C.POINTER(C.c_uint32)), ("dy", C.c_int32), ("dx", C.c_int32), ("nlimbs", C.c_int32)]


class Upoly(C.Structure):
    _fields_ = [("limbs", C.POINTER(C.c_uint32)), ("deg", C.c_int32), ("nlimbs", C.c_int32)]


class Plan(C.Structure):
    _fields_ = [("deg_bound", C.c_int32), ("out_nlimbs", C.c_int32), ("nprimes", C.c_int32),
                ("reserved", C.c_int32), ("workspace_bytes", C.c_size_t)]


_lib = None
_lib_lock = threading.Lock()


def lib():
    """Load libsnc.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} not found: build it with python -m paper_1103_4697_amd.build")
            # torch's HIP runtime libraries first: the library then binds to the
            # same runtime (identical sonames) instead of loading the system
            # copy, which would leave one of the two without a visible device
            import torch  # noqa: F401
            L = C.CDLL(LIB_PATH)
            P, I32, SZ, VP = C.POINTER, C.c_int32, C.c_size_t, C.c_void_p
            sig = {
                "snc_version": (C.c_int, []),
                "snc_status_str": (C.c_char_p, [C.c_int]),
                "snc_create": (C.c_int, [C.c_int, P(VP)]),
                "snc_destroy": (C.c_int, [VP]),
                "snc_last_error": (C.c_char_p, [VP]),
                "snc_set_timing": (C.c_int, [VP, C.c_int]),
                "snc_get_timing": (C.c_int, [VP, P(C.c_char_p), P(C.c_float), P(I32), C.c_int]),
                "snc_microbench": (C.c_int, [VP, C.c_int, I32, VP, SZ, VP, P(C.c_double)]),
                "snc_set_tuning": (C.c_int, [VP, C.c_int]),
                "snc_set_eval_variant": (C.c_int, [VP, I32, I32, I32]),
                "snc_set_gcd_variant": (C.c_int, [VP, C.c_int]),
                "snc_prepared_sqfree_degrees": (C.c_int, [VP, C.c_int, P(I32), P(I32), C.c_int]),
                "snc_get_tuning": (C.c_int, [VP, P(I32), P(C.c_float), C.c_int, P(C.c_float)]),
                "snc_prime": (C.c_uint32, [I32]),
                "snc_resultant_y_plan": (C.c_int, [P(Bipoly), P(Bipoly), P(Plan)]),
                "snc_resultant_y": (C.c_int, [VP, P(Bipoly), P(Bipoly), VP, SZ, VP, P(Upoly)]),
                "snc_resultant_y_noalloc": (C.c_int, [VP, P(Bipoly), P(Bipoly), VP, P(Upoly)]),
                "snc_resultant_y_batch_plan": (C.c_int, [I32, P(Bipoly), P(Bipoly), P(Plan), P(Plan)]),
                "snc_resultant_y_batch": (C.c_int, [VP, I32, P(Bipoly), P(Bipoly), VP, SZ, VP, P(Upoly)]),
                "snc_resultant_y_prepare": (C.c_int, [VP, I32, P(Bipoly), P(Bipoly), VP, SZ, VP, P(VP)]),
                "snc_prepared_run": (C.c_int, [VP, VP, P(Upoly)]),
                "snc_prepared_stage_bytes": (SZ, [VP]),
                "snc_prepared_submit": (C.c_int, [VP, VP, SZ, VP, P(C.c_int64)]),
                "snc_prepared_collect": (C.c_int, [VP, C.c_int64, P(Upoly)]),
                "snc_prepared_destroy": (C.c_int, [VP]),
                "snc_server_create": (C.c_int, [VP, VP, SZ, I32, I32, P(VP)]),
                "snc_submit_resultant_y": (C.c_int, [VP, P(Bipoly), P(Bipoly), P(C.c_uint64)]),
                "snc_submit_gcd_z": (C.c_int, [VP, P(Upoly), P(Upoly), P(C.c_uint64)]),
                "snc_poll": (C.c_int, [VP, C.c_uint64, P(Upoly)]),
                "snc_request_times": (C.c_int, [VP, C.c_uint64, P(C.c_double), P(C.c_double)]),
                "snc_server_wait": (C.c_int, [VP, C.c_int64, C.c_double]),
                "snc_server_destroy": (C.c_int, [VP]),
                "snc_gcd_z_plan": (C.c_int, [P(Upoly), P(Upoly), P(Plan)]),
                "snc_gcd_z": (C.c_int, [VP, P(Upoly), P(Upoly), VP, SZ, VP, P(Upoly)]),
                "snc_gcd_z_deriv_plan": (C.c_int, [P(Upoly), P(Plan)]),
                "snc_gcd_z_batch_plan": (C.c_int, [I32, P(Upoly), P(Upoly), P(Plan), P(Plan)]),
                "snc_prepared_sqfree_plan": (C.c_int, [VP, P(Plan), P(Plan)]),
                "snc_prepared_run_sqfree": (C.c_int, [VP, VP, SZ, VP, P(Upoly), P(Upoly)]),
                "snc_gcd_z_batch": (C.c_int, [VP, I32, P(Upoly), P(Upoly), VP, SZ, VP, P(Upoly)]),
                "snc_gcd_z_deriv": (C.c_int, [VP, P(Upoly), VP, SZ, VP, P(Upoly)]),
                "snc_fastlift_q_plan": (C.c_int, [P(Bipoly), P(Plan)]),
                "snc_fastlift_q": (C.c_int, [VP, P(Bipoly), VP, SZ, VP, P(Upoly)]),
                "snc_content_y_plan": (C.c_int, [P(Bipoly), P(Plan)]),
                "snc_content_y_batch_plan": (C.c_int, [I32, P(Bipoly), P(Plan), P(Plan)]),
                "snc_content_y_batch": (C.c_int, [VP, I32, P(Bipoly), VP, SZ, VP, P(Upoly)]),
                "snc_arrangement_prepare": (C.c_int, [VP, I32, P(Bipoly), VP, SZ, VP, P(VP)]),
                "snc_arrangement_plan": (C.c_int, [VP, P(Plan), P(Plan), P(Plan)]),
                "snc_arrangement_run": (C.c_int, [VP, VP, SZ, VP, P(Upoly), P(Upoly)]),
                "snc_arrangement_destroy": (C.c_int, [VP]),
                "snc_content_y": (C.c_int, [VP, P(Bipoly), VP, SZ, VP, P(Upoly)]),
                "snc_sqfree_plan": (C.c_int, [P(Upoly), P(Plan)]),
                "snc_sqfree": (C.c_int, [VP, P(Upoly), VP, SZ, VP, I32, P(C.c_uint32), P(C.c_uint32), I32,
                                         P(I32), P(I32), I32, P(I32)]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(L, name, None)
                if fn is None:
                    continue
                fn.restype = res
                fn.argtypes = args
            _lib = L
        return _lib


def _status_name(s):
    try:
        return lib().snc_status_str(s).decode()
    except Exception:
        return str(s)


# ---------------------------------------------------------------------------
# Integer marshalling (two's complement 32-bit limbs)
# ---------------------------------------------------------------------------

def _limbs_needed(vals) -> int:
    n = 1
    for v in vals:
        v = int(v)
        while not (-(1 << (32 * n - 1)) <= v < (1 << (32 * n - 1))):
            n += 1
    return n


def ints_to_limbs(vals, nl: int) -> np.ndarray:
    """Flat sequence of Python ints -> uint32 array [len][nl]."""
    vals = list(vals)
    out = np.empty((len(vals), nl), dtype=np.uint32)
    nbytes = 4 * nl
    for i, v in enumerate(vals):
        out[i] = np.frombuffer(int(v).to_bytes(nbytes, "little", signed=True), dtype="<u4")
    return out


def limbs_to_ints(arr: np.ndarray) -> list:
    """uint32 array [n][nl] -> list of Python ints."""
    arr = np.ascontiguousarray(arr, dtype=np.uint32)
    return [int.from_bytes(row.tobytes(), "little", signed=True) for row in arr]


def bivariate_limbs(F):
    """Coefficient array F[i][k] -> (uint32 limbs [dy+1][dx+1][nl], dy, dx, nl)."""
    if isinstance(F, np.ndarray) and F.dtype == np.int64:
        A = np.ascontiguousarray(F)
        if A.size == 0:
            return None, -1, -1, 1
        return A.view(np.uint32).reshape(A.shape[0], A.shape[1], 2), A.shape[0] - 1, A.shape[1] - 1, 2
    rows = [[int(c) for c in r] for r in F]
    if not rows:
        return None, -1, -1, 1
    dx = max((len(r) for r in rows), default=1) - 1
    dx = max(dx, 0)
    flat = []
    for r in rows:
        flat.extend(r + [0] * (dx + 1 - len(r)))
    nl = _limbs_needed(flat)
    L = ints_to_limbs(flat, nl).reshape(len(rows), dx + 1, nl)
    return L, len(rows) - 1, dx, nl


def _as_bipoly(F, keep):
    L, dy, dx, nl = bivariate_limbs(F)
    b = Bipoly()
    if L is None:
        b.limbs, b.dy, b.dx, b.nlimbs = None, -1, 0, 1
        return b
    L = np.ascontiguousarray(L, dtype=np.uint32)
    keep.append(L)
    b.limbs = L.ctypes.data_as(C.POINTER(C.c_uint32))
    b.dy, b.dx, b.nlimbs = dy, dx, nl
    return b


def _as_upoly(a, keep):
    vals = [int(c) for c in a]
    while vals and vals[-1] == 0:
        vals.pop()
    u = Upoly()
    if not vals:
        u.limbs, u.deg, u.nlimbs = None, -1, 1
        return u
    nl = _limbs_needed(vals)
    L = ints_to_limbs(vals, nl)
    keep.append(L)
    u.limbs = L.ctypes.data_as(C.POINTER(C.c_uint32))
    u.deg, u.nlimbs = len(vals) - 1, nl
    return u


def _out_upoly(deg_cap, nl, keep):
    buf = np.zeros((max(deg_cap, 0) + 1, max(nl, 1)), dtype=np.uint32)
    keep.append(buf)
    u = Upoly()
    u.limbs = buf.ctypes.data_as(C.POINTER(C.c_uint32))
    u.deg, u.nlimbs = deg_cap, max(nl, 1)
    return u, buf


def _read_upoly(u, buf):
    if u.deg < 0:
        return []
    return limbs_to_ints(buf[: u.deg + 1])


# ---------------------------------------------------------------------------
# Context and device workspace
# ---------------------------------------------------------------------------

class Context:
    """A library context on one device plus a growable device workspace
    (a torch uint8 tensor) and the stream the calls run on."""

    def __init__(self, device: int = 0):
        import torch  # device memory and streams only
        self._torch = torch
        self.device = device
        h = C.c_void_p()
        st = lib().snc_create(device, C.byref(h))
        if st != SNC_OK:
            raise SncError(st, "snc_create failed")
        self.h = h
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            lib().snc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return lib().snc_last_error(self.h).decode()

    def workspace(self, nbytes: int):
        torch = self._torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def stream_handle(self, stream=None):
        torch = self._torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def check(self, st, what):
        if st != SNC_OK:
            raise SncError(st, f"{what}: {self.error()}")

    def set_timing(self, on: bool):
        lib().snc_set_timing(self.h, 1 if on else 0)

    def microbench(self, kind: str, iters: int = 4096) -> float:
        """Measured operations/s of one integer operation over the whole
        device: kind 'montgomery', 'mul_lo' or 'mad_u64' (snc_microbench)."""
        kinds = {"montgomery": 0, "mul_lo": 1, "mad_u64": 2}
        props = self._torch.cuda.get_device_properties(self.device)
        ws = self.workspace(props.multi_processor_count * 64 * 16 * 4)
        rate = C.c_double(0.0)
        st = lib().snc_microbench(self.h, kinds[kind], iters, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                                  self.stream_handle(), C.byref(rate))
        self.check(st, "snc_microbench")
        return rate.value

    def set_tuning(self, mode: int):
        """Evaluation autotuner: 0 off, 1 tune untuned classes (default), 2 retune."""
        self.check(lib().snc_set_tuning(self.h, mode), "snc_set_tuning")

    def set_gcd_variant(self, variant: int):
        """Euclid of the square-free check: 0 automatic, 1 one wavefront per
        (pair, prime), 2 the blocked Euclid (a workgroup per (pair, prime))
        wherever it applies (snc_set_gcd_variant)."""
        self.check(lib().snc_set_gcd_variant(self.h, variant), "snc_set_gcd_variant")

    def set_eval_variant(self, class_cap: int, wpe: int, chunk: int = 0):
        """Force the evaluation kernel variant of a register class (wpe 0 clears)."""
        self.check(lib().snc_set_eval_variant(self.h, class_cap, wpe, chunk), "snc_set_eval_variant")

    def tuning(self):
        """The last batched preparation's evaluation variants, one dict per class."""
        cap = 8
        info = (C.c_int32 * (6 * cap))()
        ms = (C.c_float * (2 * cap))()
        tms = C.c_float(0.0)
        n = lib().snc_get_tuning(self.h, info, ms, cap, C.byref(tms))
        src = {0: "default", 1: "measured", 2: "cached", 3: "forced"}
        out = []
        for i in range(min(n, cap)):
            o = info[6 * i: 6 * i + 6]
            out.append({"class": o[0], "wpe": o[1], "chunk": o[2], "grid": o[3], "source": src.get(o[4], o[4]),
                        "candidates": o[5], "best_ms": round(ms[2 * i], 4), "default_ms": round(ms[2 * i + 1], 4)})
        return out, float(tms.value)

    def timing(self):
        cap = 32
        names = (C.c_char_p * cap)()
        ms = (C.c_float * cap)()
        launches = (C.c_int32 * cap)()
        n = lib().snc_get_timing(self.h, names, ms, launches, cap)
        return [(names[i].decode(), float(ms[i]), int(launches[i])) for i in range(min(n, cap))]


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


# ---------------------------------------------------------------------------
# Resultants
# ---------------------------------------------------------------------------

def resultant_plan(f, g) -> Plan:
    keep = []
    bf, bg = _as_bipoly(f, keep), _as_bipoly(g, keep)
    p = Plan()
    st = lib().snc_resultant_y_plan(C.byref(bf), C.byref(bg), C.byref(p))
    if st != SNC_OK:
        raise SncError(st, "snc_resultant_y_plan")
    return p


def resultant_y(f, g, ctx: Context | None = None, stream=None) -> list:
    """res_y(f, g) in Z[x] as an ascending list of Python ints ([] for 0)."""
    ctx = ctx or default_context()
    keep = []
    bf, bg = _as_bipoly(f, keep), _as_bipoly(g, keep)
    p = Plan()
    ctx.check(lib().snc_resultant_y_plan(C.byref(bf), C.byref(bg), C.byref(p)), "plan")
    u, buf = _out_upoly(p.deg_bound, p.out_nlimbs, keep)
    ws = ctx.workspace(p.workspace_bytes)
    st = lib().snc_resultant_y(ctx.h, C.byref(bf), C.byref(bg), C.c_void_p(ws.data_ptr()),
                               C.c_size_t(ws.numel()), ctx.stream_handle(stream), C.byref(u))
    ctx.check(st, "snc_resultant_y")
    return _read_upoly(u, buf)


def resultant_y_noalloc(f, g, ctx: Context | None = None, stream=None) -> list:
    """res_y(f, g) through snc_resultant_y_noalloc: the library's fixed
    device scratch array instead of a workspace (no device allocation)."""
    ctx = ctx or default_context()
    keep = []
    bf, bg = _as_bipoly(f, keep), _as_bipoly(g, keep)
    p = Plan()
    ctx.check(lib().snc_resultant_y_plan(C.byref(bf), C.byref(bg), C.byref(p)), "plan")
    u, buf = _out_upoly(p.deg_bound, p.out_nlimbs, keep)
    st = lib().snc_resultant_y_noalloc(ctx.h, C.byref(bf), C.byref(bg), ctx.stream_handle(stream), C.byref(u))
    ctx.check(st, "snc_resultant_y_noalloc")
    return _read_upoly(u, buf)


NOALLOC_SCRATCH_BYTES = 64 << 20  # SNC_NOALLOC_SCRATCH_BYTES of snc.h


class ResultantBatch:
    """A prepared batch of resultants: planned and uploaded once into a device
    workspace owned by this object, then run any number of times (the device
    pipeline is captured as a HIP graph on the first run and replayed)."""

    def __init__(self, pairs, ctx: Context | None = None, stream=None):
        import torch
        self.ctx = ctx or default_context()
        self.keep = []
        n = len(pairs)
        self.n = n
        self.F = (Bipoly * n)()
        self.G = (Bipoly * n)()
        for i, (f, g) in enumerate(pairs):
            self.F[i] = _as_bipoly(f, self.keep)
            self.G[i] = _as_bipoly(g, self.keep)
        each = (Plan * n)()
        total = Plan()
        st = lib().snc_resultant_y_batch_plan(n, self.F, self.G, each, C.byref(total))
        if st != SNC_OK:
            raise SncError(st, "snc_resultant_y_batch_plan")
        self.plan = total
        self.each = each
        self.out = (Upoly * n)()
        self.bufs = []
        self.caps = []
        for i in range(n):
            u, buf = _out_upoly(each[i].deg_bound, each[i].out_nlimbs, self.keep)
            self.out[i] = u
            self.bufs.append(buf)
            self.caps.append((each[i].deg_bound, each[i].out_nlimbs))
        self.ws = torch.empty(max(total.workspace_bytes, 256), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        h = C.c_void_p()
        st = lib().snc_resultant_y_prepare(self.ctx.h, n, self.F, self.G, C.c_void_p(self.ws.data_ptr()),
                                           C.c_size_t(self.ws.numel()), self.ctx.stream_handle(stream), C.byref(h))
        self.ctx.check(st, "snc_resultant_y_prepare")
        self.h = h

    def run(self, stream=None):
        for i, (d, nl) in enumerate(self.caps):
            self.out[i].deg = d
            self.out[i].nlimbs = nl
        st = lib().snc_prepared_run(self.h, self.ctx.stream_handle(stream), self.out)
        self.ctx.check(st, "snc_prepared_run")

    def submit(self, stream=None) -> int:
        """Enqueue one run and the download of its results
        (snc_prepared_submit, device staging in a tensor owned by this
        object); returns its ticket.  The next submit's kernels overlap this
        run's download.  At most two runs are outstanding."""
        import torch
        if not hasattr(self, "stage"):
            nb = lib().snc_prepared_stage_bytes(self.h)
            self.stage = torch.empty(max(nb, 256), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        t = C.c_int64(-1)
        self.ctx.check(lib().snc_prepared_submit(self.h, C.c_void_p(self.stage.data_ptr()),
                                                 C.c_size_t(self.stage.numel()), self.ctx.stream_handle(stream),
                                                 C.byref(t)), "snc_prepared_submit")
        return t.value

    def collect(self, ticket: int):
        """Wait for a submitted run and write its results into the output
        buffers (read them with results())."""
        for i, (d, nl) in enumerate(self.caps):
            self.out[i].deg = d
            self.out[i].nlimbs = nl
        self.ctx.check(lib().snc_prepared_collect(self.h, C.c_int64(ticket), self.out), "snc_prepared_collect")

    def run_sqfree(self, stream=None):
        """Run the pipeline and gcd(R_i, R_i') in the same pass
        (snc_prepared_run_sqfree): the resultants land in bufs/out as with
        run(), the gcds in gbufs/gout (read them with sqfree_results)."""
        import torch
        if not hasattr(self, "gout"):
            n = self.n
            each = (Plan * n)()
            total = Plan()
            self.ctx.check(lib().snc_prepared_sqfree_plan(self.h, each, C.byref(total)), "snc_prepared_sqfree_plan")
            self.gout = (Upoly * n)()
            self.gbufs, self.gcaps = [], []
            for i in range(n):
                u, buf = _out_upoly(each[i].deg_bound, each[i].out_nlimbs, self.keep)
                self.gout[i] = u
                self.gbufs.append(buf)
                self.gcaps.append((each[i].deg_bound, each[i].out_nlimbs))
            self.gws = torch.empty(max(total.workspace_bytes, 256), dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        for i, (d, nl) in enumerate(self.caps):
            self.out[i].deg = d
            self.out[i].nlimbs = nl
        for i, (d, nl) in enumerate(self.gcaps):
            self.gout[i].deg = d
            self.gout[i].nlimbs = nl
        st = lib().snc_prepared_run_sqfree(self.h, C.c_void_p(self.gws.data_ptr()), C.c_size_t(self.gws.numel()),
                                           self.ctx.stream_handle(stream), self.out, self.gout)
        self.ctx.check(st, "snc_prepared_run_sqfree")

    def sqfree_results(self):
        return [_read_upoly(self.gout[i], self.gbufs[i]) for i in range(self.n)]

    def degrees(self):
        return [self.out[i].deg for i in range(self.n)]

    def sqfree_degrees(self, i: int):
        """After run_sqfree: (d, e) for pair i over its primes, d[q] = deg R
        mod p_q and e[q] = deg gcd(R, R') mod p_q (snc_prepared_sqfree_degrees)."""
        k = lib().snc_prepared_sqfree_degrees(self.h, i, None, None, 0)
        if k < 0:
            raise SncError(k, "snc_prepared_sqfree_degrees")
        d = (C.c_int32 * max(k, 1))()
        e = (C.c_int32 * max(k, 1))()
        if k:
            st = lib().snc_prepared_sqfree_degrees(self.h, i, d, e, k)
            if st < 0:
                raise SncError(st, "snc_prepared_sqfree_degrees")
        return list(d)[:k], list(e)[:k]

    def results(self):
        return [_read_upoly(self.out[i], self.bufs[i]) for i in range(self.n)]

    def close(self):
        if getattr(self, "h", None):
            lib().snc_prepared_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlainResultants:
    """The plain form of a list of resultants: one snc_resultant_y call per
    pair (plan, upload, one pipeline of launches, download; synchronised per
    pair, no graph, nothing shared between pairs).  Inputs are marshalled
    and outputs sized once, so run() times only the library calls."""

    def __init__(self, pairs, ctx: Context | None = None, stream=None):
        self.ctx = ctx or default_context()
        self.keep = []
        self.args = []
        need = 256
        for f, g in pairs:
            bf, bg = _as_bipoly(f, self.keep), _as_bipoly(g, self.keep)
            p = Plan()
            self.ctx.check(lib().snc_resultant_y_plan(C.byref(bf), C.byref(bg), C.byref(p)), "plan")
            u, buf = _out_upoly(p.deg_bound, p.out_nlimbs, self.keep)
            self.args.append((bf, bg, u, buf, p.deg_bound, max(p.out_nlimbs, 1)))
            need = max(need, p.workspace_bytes)
        self.ws = self.ctx.workspace(need)
        self.stream = self.ctx.stream_handle(stream)

    def run(self):
        L, h, wsp, wsn = lib(), self.ctx.h, C.c_void_p(self.ws.data_ptr()), C.c_size_t(self.ws.numel())
        for bf, bg, u, _buf, d, nl in self.args:
            u.deg, u.nlimbs = d, nl
            st = L.snc_resultant_y(h, C.byref(bf), C.byref(bg), wsp, wsn, self.stream, C.byref(u))
            if st != SNC_OK:
                self.ctx.check(st, "snc_resultant_y")

    def results(self):
        return [_read_upoly(u, buf) for _bf, _bg, u, buf, _d, _nl in self.args]


def resultant_y_batch(pairs, ctx: Context | None = None, stream=None) -> list:
    """n resultants in one submission (every stage launched once over all
    pairs, as one HIP graph)."""
    ctx = ctx or default_context()
    keep = []
    n = len(pairs)
    F = (Bipoly * n)()
    G = (Bipoly * n)()
    for i, (f, g) in enumerate(pairs):
        F[i] = _as_bipoly(f, keep)
        G[i] = _as_bipoly(g, keep)
    each = (Plan * n)()
    total = Plan()
    ctx.check(lib().snc_resultant_y_batch_plan(n, F, G, each, C.byref(total)), "batch plan")
    out = (Upoly * n)()
    bufs = []
    for i in range(n):
        u, buf = _out_upoly(each[i].deg_bound, each[i].out_nlimbs, keep)
        out[i] = u
        bufs.append(buf)
    ws = ctx.workspace(total.workspace_bytes)
    st = lib().snc_resultant_y_batch(ctx.h, n, F, G, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                                     ctx.stream_handle(stream), out)
    ctx.check(st, "snc_resultant_y_batch")
    return [_read_upoly(out[i], bufs[i]) for i in range(n)]


# ---------------------------------------------------------------------------
# gcd in Z[x]
# ---------------------------------------------------------------------------

def _limbs_upoly(x: np.ndarray):
    """Upoly view of a uint32 [deg+1][nl] limb array (rows ascending)."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    u = Upoly()
    if x.ndim != 2 or x.shape[0] == 0:
        u.limbs, u.deg, u.nlimbs = None, -1, 1
    else:
        u.limbs = x.ctypes.data_as(C.POINTER(C.c_uint32))
        u.deg, u.nlimbs = x.shape[0] - 1, x.shape[1]
    return u, x


def _run_gcd(ctx: Context, run, plan):
    """Call a gcd entry point with the context's workspace and a cached output
    buffer; the plan is asked only when the call reports that the workspace
    (SNC_ENOMEM) or the output (SNC_ERANGE) is too small.  Returns the result
    rows as a fresh uint32 [deg+1][nl] array."""
    buf = getattr(ctx, "_gcd_buf", None)
    ws = ctx._ws
    if buf is None or ws is None:
        p = Plan()
        ctx.check(plan(p), "gcd plan")
        buf = np.zeros((max(p.deg_bound, 0) + 1, max(p.out_nlimbs, 1)), dtype=np.uint32)
        ws = ctx.workspace(p.workspace_bytes)
    for _ in range(3):
        u = Upoly()
        u.limbs = buf.ctypes.data_as(C.POINTER(C.c_uint32))
        u.deg, u.nlimbs = buf.shape[0] - 1, buf.shape[1]
        st = run(ws, u)
        if st == SNC_OK:
            ctx._gcd_buf = buf
            return buf[: u.deg + 1].copy()
        if st == SNC_ERANGE:
            buf = np.zeros((max(u.deg, buf.shape[0] - 1) + 1, max(u.nlimbs, buf.shape[1])), dtype=np.uint32)
        elif st == SNC_ENOMEM:
            p = Plan()
            ctx.check(plan(p), "gcd plan")
            ws = ctx.workspace(p.workspace_bytes)
        else:
            break
    ctx.check(st, "gcd")
    raise SncError(st, "gcd: sizes did not settle")


def gcd_z_limbs(a_limbs: np.ndarray, b_limbs: np.ndarray, ctx: Context | None = None, stream=None):
    """gcd on limb arrays (uint32 [deg+1][nl], two's complement): returns the
    result as a uint32 [deg+1][nl] array (empty for the zero polynomial)."""
    ctx = ctx or default_context()
    ua, a_limbs = _limbs_upoly(a_limbs)
    ub, b_limbs = _limbs_upoly(b_limbs)
    sh = ctx.stream_handle(stream)
    return _run_gcd(ctx,
                    lambda ws, u: lib().snc_gcd_z(ctx.h, C.byref(ua), C.byref(ub), C.c_void_p(ws.data_ptr()),
                                                  C.c_size_t(ws.numel()), sh, C.byref(u)),
                    lambda p: lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p)))


def gcd_z(a, b, ctx: Context | None = None, stream=None) -> list:
    """gcd(a, b) in Z[x] (content kept, positive leading coefficient)."""
    ctx = ctx or default_context()
    keep = []
    ua, ub = _as_upoly(a, keep), _as_upoly(b, keep)
    sh = ctx.stream_handle(stream)
    rows = _run_gcd(ctx,
                    lambda ws, u: lib().snc_gcd_z(ctx.h, C.byref(ua), C.byref(ub), C.c_void_p(ws.data_ptr()),
                                                  C.c_size_t(ws.numel()), sh, C.byref(u)),
                    lambda p: lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p)))
    return limbs_to_ints(rows) if len(rows) else []


def gcd_z_batch(pairs, ctx: Context | None = None, stream=None) -> list:
    """gcd(a_i, b_i) for a list of (a, b) pairs of ascending Python-int lists,
    in one batched submission (snc_gcd_z_batch)."""
    ctx = ctx or default_context()
    n = len(pairs)
    if n == 0:
        return []
    keep = []
    A = (Upoly * n)()
    B = (Upoly * n)()
    for i, (a, b) in enumerate(pairs):
        A[i] = _as_upoly(a, keep)
        B[i] = _as_upoly(b, keep)
    each = (Plan * n)()
    total = Plan()
    ctx.check(lib().snc_gcd_z_batch_plan(n, A, B, each, C.byref(total)), "gcd batch plan")
    out = (Upoly * n)()
    bufs = []
    for i in range(n):
        u, buf = _out_upoly(each[i].deg_bound, each[i].out_nlimbs, keep)
        out[i] = u
        bufs.append(buf)
    ws = ctx.workspace(total.workspace_bytes)
    st = lib().snc_gcd_z_batch(ctx.h, n, A, B, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                               ctx.stream_handle(stream), out)
    ctx.check(st, "snc_gcd_z_batch")
    return [_read_upoly(out[i], bufs[i]) for i in range(n)]


def gcd_z_deriv_limbs(a_limbs: np.ndarray, ctx: Context | None = None, stream=None):
    """gcd(a, a') on a limb array (the derivative is formed in the library)."""
    ctx = ctx or default_context()
    ua, a_limbs = _limbs_upoly(a_limbs)
    sh = ctx.stream_handle(stream)
    return _run_gcd(ctx,
                    lambda ws, u: lib().snc_gcd_z_deriv(ctx.h, C.byref(ua), C.c_void_p(ws.data_ptr()),
                                                        C.c_size_t(ws.numel()), sh, C.byref(u)),
                    lambda p: lib().snc_gcd_z_deriv_plan(C.byref(ua), C.byref(p)))


def gcd_z_deriv(a, ctx: Context | None = None, stream=None) -> list:
    """gcd(a, a') in Z[x] for a list of Python ints (ascending)."""
    ctx = ctx or default_context()
    keep = []
    ua = _as_upoly(a, keep)
    sh = ctx.stream_handle(stream)
    rows = _run_gcd(ctx,
                    lambda ws, u: lib().snc_gcd_z_deriv(ctx.h, C.byref(ua), C.c_void_p(ws.data_ptr()),
                                                        C.c_size_t(ws.numel()), sh, C.byref(u)),
                    lambda p: lib().snc_gcd_z_deriv_plan(C.byref(ua), C.byref(p)))
    return limbs_to_ints(rows) if len(rows) else []


def content_y(f, ctx: Context | None = None, stream=None) -> list:
    """Content of f in y (snc_content_y): gcd of its rows f_i(x) in Z[x] with
    a positive leading coefficient, as an ascending list of Python ints
    ([] for f = 0)."""
    ctx = ctx or default_context()
    keep = []
    bf = _as_bipoly(f, keep)
    p = Plan()
    ctx.check(lib().snc_content_y_plan(C.byref(bf), C.byref(p)), "snc_content_y_plan")
    u, buf = _out_upoly(p.deg_bound, p.out_nlimbs, keep)
    sh = ctx.stream_handle(stream)
    need = p.workspace_bytes
    for _ in range(3):
        ws = ctx.workspace(need)
        st = lib().snc_content_y(ctx.h, C.byref(bf), C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), sh,
                                 C.byref(u))
        if st != SNC_ENOMEM:
            break
        need = 4 * max(need, ws.numel())
    ctx.check(st, "snc_content_y")
    return _read_upoly(u, buf)


def content_y_batch(curves, ctx: Context | None = None, stream=None) -> list:
    """Contents in y of several curves (snc_content_y_batch): one tree of
    batched row gcds over all curves; a list of ascending coefficient lists."""
    ctx = ctx or default_context()
    keep = []
    n = len(curves)
    F = (Bipoly * n)()
    for i, f in enumerate(curves):
        F[i] = _as_bipoly(f, keep)
    each = (Plan * n)()
    tot = Plan()
    ctx.check(lib().snc_content_y_batch_plan(n, F, each, C.byref(tot)), "snc_content_y_batch_plan")
    out = (Upoly * n)()
    bufs = []
    for i in range(n):
        u, buf = _out_upoly(each[i].deg_bound, each[i].out_nlimbs, keep)
        out[i] = u
        bufs.append(buf)
    sh = ctx.stream_handle(stream)
    need = tot.workspace_bytes
    for _ in range(3):
        ws = ctx.workspace(need)
        st = lib().snc_content_y_batch(ctx.h, n, F, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), sh, out)
        if st != SNC_ENOMEM:
            break
        need = 4 * max(need, ws.numel())
    ctx.check(st, "snc_content_y_batch")
    return [_read_upoly(out[i], bufs[i]) for i in range(n)]


class Arrangement:
    """The projection phase of an arrangement of curves (snc_arrangement_*):
    contents of all curves in one tree of batched gcds and the primitive
    parts at construction, then every res_y(p_i, dp_i/dy) and every
    res_y(p_i, p_j), i < j, as one prepared batch per run()."""

    def __init__(self, curves, ctx: Context | None = None, stream=None):
        import torch
        self.ctx = ctx or default_context()
        self.keep = []
        n = len(curves)
        self.n = n
        F = (Bipoly * n)()
        for i, f in enumerate(curves):
            F[i] = _as_bipoly(f, self.keep)
        each = (Plan * n)()
        tot = Plan()
        self.ctx.check(lib().snc_content_y_batch_plan(n, F, each, C.byref(tot)), "snc_content_y_batch_plan")
        sh = self.ctx.stream_handle(stream)
        need = tot.workspace_bytes
        h = C.c_void_p()
        for _ in range(3):
            cws = self.ctx.workspace(need)
            st = lib().snc_arrangement_prepare(self.ctx.h, n, F, C.c_void_p(cws.data_ptr()), C.c_size_t(cws.numel()),
                                               sh, C.byref(h))
            if st != SNC_ENOMEM:
                break
            need = 4 * max(need, cws.numel())
        self.ctx.check(st, "snc_arrangement_prepare")
        self.h = h
        npairs = n + n * (n - 1) // 2
        self.npairs = npairs
        ce = (Plan * n)()
        re = (Plan * npairs)()
        rt = Plan()
        self.ctx.check(lib().snc_arrangement_plan(self.h, ce, re, C.byref(rt)), "snc_arrangement_plan")
        self.cout = (Upoly * n)()
        self.cbufs, self.ccaps = [], []
        for i in range(n):
            u, buf = _out_upoly(ce[i].deg_bound, ce[i].out_nlimbs, self.keep)
            self.cout[i] = u
            self.cbufs.append(buf)
            self.ccaps.append((ce[i].deg_bound, ce[i].out_nlimbs))
        self.rout = (Upoly * npairs)()
        self.rbufs, self.rcaps = [], []
        for i in range(npairs):
            u, buf = _out_upoly(re[i].deg_bound, re[i].out_nlimbs, self.keep)
            self.rout[i] = u
            self.rbufs.append(buf)
            self.rcaps.append((re[i].deg_bound, re[i].out_nlimbs))
        self.plan = rt
        self.ws = torch.empty(max(rt.workspace_bytes, 256), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")

    def run(self, stream=None):
        for u, (d, nl) in zip(self.cout, self.ccaps):
            u.deg, u.nlimbs = d, nl
        for u, (d, nl) in zip(self.rout, self.rcaps):
            u.deg, u.nlimbs = d, nl
        st = lib().snc_arrangement_run(self.h, C.c_void_p(self.ws.data_ptr()), C.c_size_t(self.ws.numel()),
                                       self.ctx.stream_handle(stream), self.cout, self.rout)
        self.ctx.check(st, "snc_arrangement_run")

    def contents(self):
        return [_read_upoly(self.cout[i], self.cbufs[i]) for i in range(self.n)]

    def resultants(self):
        """res_y(p_i, dp_i/dy) for each curve, then res_y(p_i, p_j) for i < j."""
        return [_read_upoly(self.rout[i], self.rbufs[i]) for i in range(self.npairs)]

    def close(self):
        if getattr(self, "h", None):
            lib().snc_arrangement_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fastlift_q(f, ctx: Context | None = None, stream=None) -> list:
    """FastLift's Q = res_y(f_x / h, f_y / h), h = gcd(f_x, f_y)
    (snc_fastlift_q), as an ascending list of Python ints; raises SncError
    with SNC_ENOTSUP when h depends on y."""
    ctx = ctx or default_context()
    keep = []
    bf = _as_bipoly(f, keep)
    p = Plan()
    ctx.check(lib().snc_fastlift_q_plan(C.byref(bf), C.byref(p)), "snc_fastlift_q_plan")
    deg, nl, need = p.deg_bound, p.out_nlimbs, p.workspace_bytes
    sh = ctx.stream_handle(stream)
    for _ in range(3):
        u, buf = _out_upoly(deg, nl, keep)
        ws = ctx.workspace(need)
        st = lib().snc_fastlift_q(ctx.h, C.byref(bf), C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), sh,
                                  C.byref(u))
        if st == SNC_ERANGE:
            deg, nl = max(deg, u.deg), max(nl, u.nlimbs)
        elif st == SNC_ENOMEM:
            need = 4 * max(need, ws.numel())
        else:
            break
    ctx.check(st, "snc_fastlift_q")
    return _read_upoly(u, buf)


def sqfree_factor(a, ctx: Context | None = None, stream=None):
    """Square-free factorisation of a in Z[x] (snc_sqfree, Yun's algorithm):
    returns (content, [(f_1, m_1), (f_2, m_2), ...]) with
    a = content * prod f_i^m_i, the f_i primitive with positive leading
    coefficients, square-free and pairwise coprime, m_1 < m_2 < ...
    (polynomials as lists of Python ints, ascending)."""
    ctx = ctx or default_context()
    keep = []
    ua = _as_upoly(a, keep)
    p = Plan()
    ctx.check(lib().snc_sqfree_plan(C.byref(ua), C.byref(p)), "snc_sqfree_plan")
    d, nl = max(p.deg_bound, 0), max(p.out_nlimbs, 1)
    cap, maxf = 2 * d + 1, max(d, 1)
    content = np.zeros(nl, dtype=np.uint32)
    limbs = np.zeros((cap, nl), dtype=np.uint32)
    degs = np.zeros(maxf, dtype=np.int32)
    mults = np.zeros(maxf, dtype=np.int32)
    nf = C.c_int32(0)
    sh = ctx.stream_handle(stream)
    U32, I32 = C.POINTER(C.c_uint32), C.POINTER(C.c_int32)
    need = p.workspace_bytes
    for _ in range(3):
        ws = ctx.workspace(need)
        st = lib().snc_sqfree(ctx.h, C.byref(ua), C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()), sh, nl,
                              content.ctypes.data_as(U32), limbs.ctypes.data_as(U32), cap,
                              degs.ctypes.data_as(I32), mults.ctypes.data_as(I32), maxf, C.byref(nf))
        if st != SNC_ENOMEM:
            break
        need = 4 * max(need, ws.numel())
    ctx.check(st, "snc_sqfree")
    out, pos = [], 0
    for i in range(nf.value):
        n = int(degs[i]) + 1
        out.append((limbs_to_ints(limbs[pos:pos + n]), int(mults[i])))
        pos += n
    return limbs_to_ints(content[None, :])[0], out


class Server:
    """Request loop with continuous batching (snc_server_*): submit resultant
    and gcd jobs as they arrive, poll their results."""

    def __init__(self, pool_bytes: int = 1 << 30, max_slots: int = 64, nstreams: int = 4,
                 ctx: Context | None = None):
        import torch
        self.ctx = ctx or default_context()
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        torch.cuda.synchronize()
        h = C.c_void_p()
        st = lib().snc_server_create(self.ctx.h, C.c_void_p(self.pool.data_ptr()), C.c_size_t(pool_bytes),
                                     max_slots, nstreams, C.byref(h))
        if st != SNC_OK:
            raise SncError(st, "snc_server_create")
        self.h = h
        self._caps = {}

    def submit_resultant(self, f, g) -> int:
        keep = []
        bf, bg = _as_bipoly(f, keep), _as_bipoly(g, keep)
        t = C.c_uint64()
        st = lib().snc_submit_resultant_y(self.h, C.byref(bf), C.byref(bg), C.byref(t))
        if st != SNC_OK:
            raise SncError(st, "snc_submit_resultant_y")
        p = Plan()
        lib().snc_resultant_y_plan(C.byref(bf), C.byref(bg), C.byref(p))
        self._caps[t.value] = (p.deg_bound, p.out_nlimbs)
        return t.value

    def submit_gcd(self, a, b) -> int:
        keep = []
        ua, ub = _as_upoly(a, keep), _as_upoly(b, keep)
        t = C.c_uint64()
        st = lib().snc_submit_gcd_z(self.h, C.byref(ua), C.byref(ub), C.byref(t))
        if st != SNC_OK:
            raise SncError(st, "snc_submit_gcd_z")
        p = Plan()
        lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p))
        self._caps[t.value] = (p.deg_bound, p.out_nlimbs)
        return t.value

    def poll(self, ticket: int):
        """The result as a list of ints, or None while it is not finished."""
        d, nl = self._caps[ticket]
        keep = []
        u, buf = _out_upoly(d, nl, keep)
        st = lib().snc_poll(self.h, C.c_uint64(ticket), C.byref(u))
        if st == SNC_EAGAIN:
            return None
        if st != SNC_OK:
            raise SncError(st, "snc_poll")
        self._caps.pop(ticket, None)
        return _read_upoly(u, buf)

    def times(self, ticket: int):
        s, d = C.c_double(), C.c_double()
        st = lib().snc_request_times(self.h, C.c_uint64(ticket), C.byref(s), C.byref(d))
        if st != SNC_OK:
            return None
        return s.value, d.value

    def wait(self, completed: int, timeout_s: float = 60.0) -> bool:
        return lib().snc_server_wait(self.h, completed, timeout_s) == SNC_OK

    def close(self):
        if getattr(self, "h", None):
            lib().snc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prime(i: int) -> int:
    return int(lib().snc_prime(i))
