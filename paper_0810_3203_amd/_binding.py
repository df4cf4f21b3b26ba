"""ctypes binding of libtft.so with the C names of include/tft.h.

Device buffers are torch tensors (their data_ptr() is passed through); streams
are torch streams (cuda_stream handle), defaulting to the current stream.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libtft.so")

FERMAT = 1
NEGA = 2
PRIME = 3
PRIME_P = 15 * (1 << 27) + 1  # the word-size prime of the Z/pZ ring

_STATUS_NAMES = {0: "TFT_OK", 1: "TFT_E_ARG", 2: "TFT_E_RING", 3: "TFT_E_RANGE", 4: "TFT_E_WORKSPACE",
                 5: "TFT_E_DEVICE", 6: "TFT_E_UNSUPPORTED"}


class TFTError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, status_string(status), _STATUS_NAMES.get(status, status)))


class Ring(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("N", ctypes.c_uint32), ("K", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("m", ctypes.c_uint64)]

    def __repr__(self):
        if self.kind == FERMAT:
            return "Ring(Z/(2^%d+1))" % self.N
        return "Ring((Z/%dZ)[y]/(y^%d+1))" % (self.m, self.K)


# top_l1 value selecting L1 = 2 at every level above the leaf (TFT_SPLIT_DC)
SPLIT_DC = 0xFFFFFFFF
POLICY_GIVEN, POLICY_RULE, POLICY_MODEL = 0, 1, 2


class Split(ctypes.Structure):
    _fields_ = [("top_l1", ctypes.c_uint32), ("leaf_log2", ctypes.c_uint32)]


class SSTiming(ctypes.Structure):
    _fields_ = [("pack_ms", ctypes.c_float), ("tft_g_ms", ctypes.c_float), ("tft_h_ms", ctypes.c_float),
                ("pointwise_ms", ctypes.c_float), ("itft_ms", ctypes.c_float), ("unpack_ms", ctypes.c_float),
                ("total_ms", ctypes.c_float), ("leaf_kernel_ms", ctypes.c_float), ("leaf_launches", ctypes.c_uint32),
                ("n", ctypes.c_uint32), ("l", ctypes.c_uint32), ("N", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SSParams(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("l", ctypes.c_uint32), ("split", Split), ("k", ctypes.c_uint32),
                ("pad_rows", ctypes.c_uint32), ("zeta_exp", ctypes.c_uint32)]


class ZXRequest(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("len_g", ctypes.c_uint64), ("g_limbs", ctypes.c_uint32),
                ("h", ctypes.c_void_p), ("len_h", ctypes.c_uint64), ("h_limbs", ctypes.c_uint32),
                ("out", ctypes.c_void_p), ("out_limbs", ctypes.c_uint32), ("params", SSParams)]


SS_FEATURES = 15
STATIC_SCRATCH_BYTES = 32 << 20


def fermat_ring(N: int) -> Ring:
    return Ring(FERMAT, N, 0, 0, 0)


def nega_ring(K: int, m: int) -> Ring:
    return Ring(NEGA, 0, K, 0, m)


def prime_ring() -> Ring:
    """Z/pZ, p = 15 2^27 + 1 (the small-coefficient ring; cells are uint32 residues)."""
    return Ring(PRIME, 0, 0, 0, PRIME_P)


_lib = None


def lib():
    """The loaded libtft.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise ImportError("libtft.so not built: run `python -m paper_0810_3203_amd.build` "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(lib_path)
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        RP = ctypes.POINTER(Ring)
        L.tft_status_string.argtypes = [I]
        L.tft_status_string.restype = ctypes.c_char_p
        L.tft_last_error.argtypes = []
        L.tft_last_error.restype = ctypes.c_char_p
        L.tft_ring_check.argtypes = [RP]
        L.tft_ring_check.restype = I
        L.tft_elem_bytes.argtypes = [RP]
        L.tft_elem_bytes.restype = U64
        L.tft_array_bytes.argtypes = [RP, U64]
        L.tft_array_bytes.restype = U64
        L.tft_transform_workspace.argtypes = [RP, U32, U32, U64, U64, U64, U32, ctypes.POINTER(U64)]
        L.tft_transform_workspace.restype = I
        L.tft_forward.argtypes = [RP, U32, U64, U64, U64, P, P, U64, P]
        L.tft_forward.restype = I
        L.itft_inverse.argtypes = [RP, U32, U64, U64, U64, U32, P, P, U64, P]
        L.itft_inverse.restype = I
        L.tft_alu_rate.argtypes = [U32, U32, U32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(U64),
                                   ctypes.POINTER(ctypes.c_double), P]
        L.tft_alu_rate.restype = I
        L.tft_debug_base_cases.argtypes = [RP, U32, P, P, P]
        L.tft_debug_base_cases.restype = I
        L.pointwise_mul.argtypes = [RP, U64, P, P, P, U64, U32, P]
        L.pointwise_mul.restype = I
        L.zx_mul_ss_workspace.argtypes = [U64, U32, U64, U32, ctypes.POINTER(SSParams), ctypes.POINTER(U64)]
        L.zx_mul_ss_workspace.restype = I
        L.zx_mul_ss.argtypes = [P, U64, U32, P, U64, U32, P, U32, ctypes.POINTER(SSParams), P, U64, P]
        L.zx_mul_ss.restype = I
        L.zx_mul_ss_static.argtypes = [P, U64, U32, P, U64, U32, P, U32, ctypes.POINTER(SSParams), P]
        L.zx_mul_ss_static.restype = I
        L.zx_mul_ss_timed.argtypes = [P, U64, U32, P, U64, U32, P, U32, ctypes.POINTER(SSParams), P, U64, P,
                                      ctypes.POINTER(SSTiming)]
        L.zx_mul_ss_timed.restype = I
        L.zmx_mul_nussbaumer_workspace.argtypes = [U64, U64, U32, ctypes.POINTER(U64)]
        L.zmx_mul_nussbaumer_workspace.restype = I
        L.zpx_mul_ntt_workspace.argtypes = [U64, U64, ctypes.POINTER(U64)]
        L.zpx_mul_ntt_workspace.restype = I
        L.zpx_mul_ntt.argtypes = [P, U64, P, U64, U32, P, P, U64, P]
        L.zpx_mul_ntt.restype = I
        L.zmx_mul_nussbaumer.argtypes = [P, U64, P, U64, U64, U32, P, P, U64, P]
        L.zmx_mul_nussbaumer.restype = I
        L.tft_plan_create.argtypes = [RP, U32, U32, U64, U64, U64, U32, ctypes.POINTER(Split), ctypes.POINTER(P)]
        L.tft_plan_create.restype = I
        L.tft_plan_execute.argtypes = [P, P, P]
        L.tft_plan_execute.restype = I
        L.tft_plan_destroy.argtypes = [P]
        L.tft_plan_destroy.restype = None
        L.tft_plan_base_cases.argtypes = [P]
        L.tft_plan_base_cases.restype = U64
        L.tft_plan_export.argtypes = [P, P, U64, ctypes.POINTER(U64)]
        L.tft_plan_export.restype = I
        RQ = ctypes.POINTER(ZXRequest)
        SP = ctypes.POINTER(SSParams)
        FP = ctypes.POINTER(ctypes.c_float)
        L.tft_batch_plan_create.argtypes = [RQ, U32, U64, I, P, ctypes.POINTER(P)]
        L.tft_batch_plan_create.restype = I
        L.tft_batch_plan_params.argtypes = [P, SP]
        L.tft_batch_plan_params.restype = I
        L.tft_batch_plan_workspace.argtypes = [P]
        L.tft_batch_plan_workspace.restype = U64
        L.tft_batch_plan_status.argtypes = [P, ctypes.POINTER(I)]
        L.tft_batch_plan_status.restype = I
        L.tft_batch_plan_launches.argtypes = [P]
        L.tft_batch_plan_launches.restype = U32
        L.tft_batch_plan_execute.argtypes = [P, P, U64, I, P]
        L.tft_batch_plan_execute.restype = I
        L.tft_batch_plan_destroy.argtypes = [P]
        L.tft_batch_plan_destroy.restype = None
        L.tft_ss_candidates.argtypes = [U64, U32, U64, U32, SP, U32, ctypes.POINTER(U32)]
        L.tft_ss_candidates.restype = I
        L.tft_ss_default_params.argtypes = [U64, U32, U64, U32, SP]
        L.tft_ss_default_params.restype = I
        L.tft_ss_features.argtypes = [U64, U32, U64, U32, SP, FP]
        L.tft_ss_features.restype = I
        L.tft_ss_time.argtypes = [RQ, SP, U32, U32, P, U64, P, FP, ctypes.POINTER(U32)]
        L.tft_ss_time.restype = I
        L.tft_mlp_create.argtypes = [U32, U32, U32, U64, ctypes.POINTER(P)]
        L.tft_mlp_create.restype = I
        L.tft_mlp_param_count.argtypes = [P]
        L.tft_mlp_param_count.restype = U64
        L.tft_mlp_get_params.argtypes = [P, FP, U64]
        L.tft_mlp_get_params.restype = I
        L.tft_mlp_set_params.argtypes = [P, FP, U64]
        L.tft_mlp_set_params.restype = I
        L.tft_mlp_forward.argtypes = [P, P, U32, P, P]
        L.tft_mlp_forward.restype = I
        L.tft_mlp_gradient.argtypes = [P, P, P, U32, P, P, P]
        L.tft_mlp_gradient.restype = I
        L.tft_mlp_train.argtypes = [P, P, P, U32, U32, ctypes.c_float, FP, P]
        L.tft_mlp_train.restype = I
        L.tft_mlp_destroy.argtypes = [P]
        L.tft_mlp_destroy.restype = None
        L.tft_mlp_choose_ss.argtypes = [P, RQ, U32, P]
        L.tft_mlp_choose_ss.restype = I
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().tft_status_string(int(status)).decode()


def _check(rc, where):
    if rc != 0:
        if rc == 5:
            where = "%s [%s]" % (where, lib().tft_last_error().decode())
        raise TFTError(rc, where)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def ring_check(ring: Ring) -> int:
    return lib().tft_ring_check(ctypes.byref(ring))


def elem_bytes(ring: Ring) -> int:
    return lib().tft_elem_bytes(ctypes.byref(ring))


def array_bytes(ring: Ring, cells: int) -> int:
    return lib().tft_array_bytes(ctypes.byref(ring), cells)


def transform_workspace(ring, direction, l, s, z, n, f=0) -> int:
    """Device workspace bytes of tft_forward (direction 0) / itft_inverse (1)."""
    b = ctypes.c_uint64(0)
    _check(lib().tft_transform_workspace(ctypes.byref(ring), direction, l, s, z, n, f, ctypes.byref(b)),
           "tft_transform_workspace")
    return b.value


def _transform_ws(ring, direction, l, s, z, n, f, x, ws):
    if ws is None:
        import torch
        need = transform_workspace(ring, direction, l, s, z, n, f)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    return ws


def tft_forward(ring, l, s, z, n, x, ws=None, stream=None):
    """In-place TFT(2^l, theta^s, z, n) on cell array x (a device tensor of
    capacity 2^l).  ws: device workspace (allocated here if None)."""
    ws = _transform_ws(ring, 0, l, s, z, n, 0, x, ws)
    _check(lib().tft_forward(ctypes.byref(ring), l, s, z, n, _ptr(x), _ptr(ws), ws.numel() * ws.element_size(),
                             _stream(stream)), "tft_forward")


def itft_inverse(ring, l, s, z, n, f, x, ws=None, stream=None):
    """In-place ITFT(2^l, theta^s, z, n, f) on cell array x."""
    ws = _transform_ws(ring, 1, l, s, z, n, f, x, ws)
    _check(lib().itft_inverse(ctypes.byref(ring), l, s, z, n, f, _ptr(x), _ptr(ws),
                              ws.numel() * ws.element_size(), _stream(stream)), "itft_inverse")


def alu_rate(kind, blocks, iters, stream=None):
    """(ms, lane_ops, shader clock Hz) of the register-only issue-rate probe (tft_alu_rate)."""
    ms = ctypes.c_float(0)
    ops = ctypes.c_uint64(0)
    hz = ctypes.c_double(0)
    _check(lib().tft_alu_rate(kind, blocks, iters, ctypes.byref(ms), ctypes.byref(ops), ctypes.byref(hz),
                              _stream(stream)), "tft_alu_rate")
    return ms.value, ops.value, hz.value


def debug_base_cases(ring, ncases, cases, out, stream=None):
    """Runs single base cases on the device (records: see tft_debug_base_cases in tft.h)."""
    _check(lib().tft_debug_base_cases(ctypes.byref(ring), ncases, _ptr(cases), _ptr(out), _stream(stream)),
           "tft_debug_base_cases")


def pointwise_mul(ring, n, a, b, c, cap, scale_log2=0, stream=None):
    """c_i = a_i b_i 2^-scale_log2 for i < n (cell arrays of capacity cap)."""
    _check(lib().pointwise_mul(ctypes.byref(ring), n, _ptr(a), _ptr(b), _ptr(c), cap, scale_log2,
                               _stream(stream)), "pointwise_mul")


def zx_mul_ss_workspace(len_g, g_limbs, len_h, h_limbs, params=None) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().zx_mul_ss_workspace(len_g, g_limbs, len_h, h_limbs, ctypes.byref(params) if params else None,
                                     ctypes.byref(out)), "zx_mul_ss_workspace")
    return out.value


def zx_mul_ss(g, h, out, params=None, ws=None, stream=None):
    """u = g h in Z[x].  g: (len_g, g_limbs) uint32-valued int32 tensor on the device, h likewise,
    out: (len_g + len_h - 1, out_limbs).  ws: uint8 device tensor (allocated here if None)."""
    len_g, g_limbs = g.shape
    len_h, h_limbs = h.shape
    out_limbs = out.shape[1]
    need = zx_mul_ss_workspace(len_g, g_limbs, len_h, h_limbs, params)
    if ws is None:
        import torch
        ws = torch.empty(need, dtype=torch.uint8, device=g.device)
    _check(lib().zx_mul_ss(_ptr(g), len_g, g_limbs, _ptr(h), len_h, h_limbs, _ptr(out), out_limbs,
                           ctypes.byref(params) if params else None, _ptr(ws), ws.numel() * ws.element_size(),
                           _stream(stream)), "zx_mul_ss")
    return out


def zx_mul_ss_static(g, h, out, params=None, stream=None):
    """zx_mul_ss from the library's static device scratch (no workspace, no allocation)."""
    len_g, g_limbs = g.shape
    len_h, h_limbs = h.shape
    _check(lib().zx_mul_ss_static(_ptr(g), len_g, g_limbs, _ptr(h), len_h, h_limbs, _ptr(out), out.shape[1],
                                  ctypes.byref(params) if params else None, _stream(stream)), "zx_mul_ss_static")
    return out


def zx_mul_ss_timed(g, h, out, params=None, ws=None, stream=None):
    """zx_mul_ss that waits for completion and returns the phase times (SSTiming.as_dict())."""
    len_g, g_limbs = g.shape
    len_h, h_limbs = h.shape
    need = zx_mul_ss_workspace(len_g, g_limbs, len_h, h_limbs, params)
    if ws is None:
        import torch
        ws = torch.empty(need, dtype=torch.uint8, device=g.device)
    tm = SSTiming()
    _check(lib().zx_mul_ss_timed(_ptr(g), len_g, g_limbs, _ptr(h), len_h, h_limbs, _ptr(out), out.shape[1],
                                 ctypes.byref(params) if params else None, _ptr(ws), ws.numel() * ws.element_size(),
                                 _stream(stream), ctypes.byref(tm)), "zx_mul_ss_timed")
    return tm.as_dict()


def zmx_mul_nussbaumer_workspace(len_g, len_h, log2K) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().zmx_mul_nussbaumer_workspace(len_g, len_h, log2K, ctypes.byref(out)),
           "zmx_mul_nussbaumer_workspace")
    return out.value


def zmx_mul_nussbaumer(g, h, m, log2K, out, ws=None, stream=None):
    """u = g h in (Z/mZ)[x]; g, h, out are int64 device tensors holding values in [0, m)."""
    len_g, len_h = g.numel(), h.numel()
    need = zmx_mul_nussbaumer_workspace(len_g, len_h, log2K)
    if ws is None:
        import torch
        ws = torch.empty(need, dtype=torch.uint8, device=g.device)
    _check(lib().zmx_mul_nussbaumer(_ptr(g), len_g, _ptr(h), len_h, m, log2K, _ptr(out), _ptr(ws),
                                    ws.numel() * ws.element_size(), _stream(stream)), "zmx_mul_nussbaumer")
    return out


def zpx_mul_ntt(g, h, out, pad_rows=0, ws=None, stream=None):
    """u = g h in (Z/pZ)[x] (p = PRIME_P); g, h, out: int32 device tensors of residues."""
    len_g, len_h = g.numel(), h.numel()
    if ws is None:
        import torch
        need = ctypes.c_uint64(0)
        _check(lib().zpx_mul_ntt_workspace(len_g, len_h, ctypes.byref(need)), "zpx_mul_ntt_workspace")
        ws = torch.empty(need.value, dtype=torch.uint8, device=g.device)
    _check(lib().zpx_mul_ntt(_ptr(g), len_g, _ptr(h), len_h, pad_rows, _ptr(out), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(stream)), "zpx_mul_ntt")
    return out


class Plan:
    """An explicit transform plan (tft_plan_create / execute / destroy / export)."""

    def __init__(self, ring, direction, l, s, z, n, f=0, top_l1=0, leaf_log2=0):
        self.ring = ring
        self.l = l
        self._p = ctypes.c_void_p()
        sp = Split(top_l1, leaf_log2)
        _check(lib().tft_plan_create(ctypes.byref(ring), direction, l, s, z, n, f, ctypes.byref(sp),
                                     ctypes.byref(self._p)), "tft_plan_create")

    def execute(self, x, stream=None):
        _check(lib().tft_plan_execute(self._p, _ptr(x), _stream(stream)), "tft_plan_execute")

    @property
    def base_cases(self) -> int:
        return lib().tft_plan_base_cases(self._p)

    def export(self):
        """The schedule as a dict of lists (see tft_plan_export in tft.h)."""
        need = ctypes.c_uint64(0)
        lib().tft_plan_export(self._p, None, 0, ctypes.byref(need))
        buf = (ctypes.c_uint64 * need.value)()
        _check(lib().tft_plan_export(self._p, buf, need.value, ctypes.byref(need)), "tft_plan_export")
        w = list(buf)
        npass, njob, nprog, nstep, nop, ord_, leaf = w[1:8]
        pos = 8

        def take(count, width):
            nonlocal pos
            out = [tuple(w[pos + i * width: pos + (i + 1) * width]) for i in range(count)]
            pos += count * width
            return out
        return dict(ord=ord_, leaf_log2=leaf, passes=take(npass, 3), jobs=take(njob, 6), progs=take(nprog, 3),
                    steps=take(nstep, 2), ops=take(nop, 5))

    def close(self):
        if self._p:
            lib().tft_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def zx_request(g, h, out, params=None) -> ZXRequest:
    """A batch request over device tensors g (len_g, g_limbs), h, out (as in zx_mul_ss)."""
    r = ZXRequest(g.data_ptr(), g.shape[0], g.shape[1], h.data_ptr(), h.shape[0], h.shape[1],
                  out.data_ptr(), out.shape[1])
    if params is not None:
        r.params = params
    return r


def requests_array(reqs):
    arr = (ZXRequest * len(reqs))()
    for i, r in enumerate(reqs):
        arr[i] = r
    return arr


class BatchPlan:
    """tft_batch_plan_*: many Z[x] products planned and run together."""

    def __init__(self, reqs, max_workspace=0, policy=POLICY_GIVEN, model=None):
        self.count = len(reqs)
        self._reqs = reqs if isinstance(reqs, ctypes.Array) else requests_array(reqs)
        self._p = ctypes.c_void_p()
        _check(lib().tft_batch_plan_create(self._reqs, self.count, max_workspace, policy,
                                           model._p if model is not None else None, ctypes.byref(self._p)),
               "tft_batch_plan_create")

    def params(self):
        """The SSParams each request was planned with."""
        arr = (SSParams * max(1, self.count))()
        _check(lib().tft_batch_plan_params(self._p, arr), "tft_batch_plan_params")
        return list(arr)[:self.count]

    @property
    def workspace(self) -> int:
        return lib().tft_batch_plan_workspace(self._p)

    @property
    def launches(self) -> int:
        return lib().tft_batch_plan_launches(self._p)

    def status(self):
        st = (ctypes.c_int * max(1, self.count))()
        _check(lib().tft_batch_plan_status(self._p, st), "tft_batch_plan_status")
        return list(st)[:self.count]

    def execute(self, ws, use_graph=False, stream=None):
        _check(lib().tft_batch_plan_execute(self._p, _ptr(ws), ws.numel() * ws.element_size() if ws is not None
                                            else 0, 1 if use_graph else 0, _stream(stream)),
               "tft_batch_plan_execute")

    def close(self):
        if self._p:
            lib().tft_batch_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ss_candidates(len_g, g_limbs, len_h, h_limbs):
    n = ctypes.c_uint32(0)
    _check(lib().tft_ss_candidates(len_g, g_limbs, len_h, h_limbs, None, 0, ctypes.byref(n)), "tft_ss_candidates")
    arr = (SSParams * n.value)()
    _check(lib().tft_ss_candidates(len_g, g_limbs, len_h, h_limbs, arr, n.value, ctypes.byref(n)),
           "tft_ss_candidates")
    return list(arr)


def ss_default_params(len_g, g_limbs, len_h, h_limbs) -> SSParams:
    p = SSParams()
    _check(lib().tft_ss_default_params(len_g, g_limbs, len_h, h_limbs, ctypes.byref(p)), "tft_ss_default_params")
    return p


def ss_features(len_g, g_limbs, len_h, h_limbs, params):
    f = (ctypes.c_float * SS_FEATURES)()
    _check(lib().tft_ss_features(len_g, g_limbs, len_h, h_limbs, ctypes.byref(params), f), "tft_ss_features")
    return list(f)


def ss_time(req, cands, reps, ws, stream=None):
    """Median ms per candidate and the index of the fastest (tft_ss_time)."""
    arr = (SSParams * len(cands))(*cands)
    ms = (ctypes.c_float * len(cands))()
    best = ctypes.c_uint32(0)
    _check(lib().tft_ss_time(ctypes.byref(req), arr, len(cands), reps, _ptr(ws), ws.numel() * ws.element_size(),
                             _stream(stream), ms, ctypes.byref(best)), "tft_ss_time")
    return list(ms), best.value


class MLP:
    """tft_mlp_*: the fp32 cost model (HIP forward, backward and Adam)."""

    def __init__(self, in_features=SS_FEATURES, hidden=64, depth=3, seed=0):
        self.in_features = in_features
        self._p = ctypes.c_void_p()
        _check(lib().tft_mlp_create(in_features, hidden, depth, seed, ctypes.byref(self._p)), "tft_mlp_create")

    @property
    def param_count(self) -> int:
        return lib().tft_mlp_param_count(self._p)

    def get_params(self):
        n = self.param_count
        buf = (ctypes.c_float * n)()
        _check(lib().tft_mlp_get_params(self._p, buf, n), "tft_mlp_get_params")
        return list(buf)

    def set_params(self, values):
        n = self.param_count
        buf = (ctypes.c_float * n)(*values)
        _check(lib().tft_mlp_set_params(self._p, buf, n), "tft_mlp_set_params")

    def forward(self, x, y, stream=None):
        _check(lib().tft_mlp_forward(self._p, _ptr(x), x.shape[0], _ptr(y), _stream(stream)), "tft_mlp_forward")
        return y

    def gradient(self, x, target, grad=None, loss=None, stream=None):
        _check(lib().tft_mlp_gradient(self._p, _ptr(x), _ptr(target), x.shape[0], _ptr(grad), _ptr(loss),
                                      _stream(stream)), "tft_mlp_gradient")

    def train(self, x, target, iters, lr, stream=None) -> float:
        fl = ctypes.c_float(0)
        _check(lib().tft_mlp_train(self._p, _ptr(x), _ptr(target), x.shape[0], iters, lr, ctypes.byref(fl),
                                   _stream(stream)), "tft_mlp_train")
        return fl.value

    def choose(self, reqs, stream=None):
        """Set reqs[i].params (a ctypes ZXRequest array) to the predicted fastest candidate."""
        _check(lib().tft_mlp_choose_ss(self._p, reqs, len(reqs), _stream(stream)), "tft_mlp_choose_ss")

    def close(self):
        if self._p:
            lib().tft_mlp_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
