"""ctypes binding of libspdz (include/spdz.h): argument marshalling only.

Device buffers are torch tensors on the GPU (int64 storage holding the raw
64-bit limbs); every computation runs in the library's HIP kernels.  The
binding fails loudly when libspdz.so is missing or a call returns an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspdz.so")

P61 = (1 << 61) - 1
P127 = (1 << 127) - 1

SPDZ_OK = 0
SPDZ_MAC_REJECT = 1
SPDZ_E_TOO_LARGE = -8
NOALLOC_SCRATCH_WORDS = 1 << 22   # SPDZ_NOALLOC_SCRATCH_WORDS of spdz.h


class SpdzError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({status})")


class Shares(ctypes.Structure):
    _fields_ = [("val", ctypes.c_void_p), ("mac", ctypes.c_void_p), ("len", ctypes.c_int64),
                ("party_stride", ctypes.c_int64), ("limb_stride", ctypes.c_int64)]


class Triple(ctypes.Structure):
    _fields_ = [("a", Shares), ("b", Shares), ("c", Shares)]


class Shares32(ctypes.Structure):
    _fields_ = [("val", ctypes.c_void_p), ("mac", ctypes.c_void_p), ("len", ctypes.c_int64),
                ("party_stride", ctypes.c_int64)]


class Triple32(ctypes.Structure):
    _fields_ = [("a", Shares32), ("b", Shares32), ("c", Shares32)]


u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libspdz.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libspdz.so not built at {LIB_PATH}: run python -m paper_2512_11112_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        sig = {
            "spdz_status_str": (ctypes.c_char_p, [i32]),
            "spdz_ctx_create": (i32, [ctypes.POINTER(vp), i32, u64p, i32, u64p, ctypes.c_uint64, vp]),
            "spdz_ctx_destroy": (i32, [vp]),
            "spdz_opened_count": (i64, [vp]),
            "spdz_ctx_set_validation": (i32, [vp, i32]),
            "spdz_open": (i32, [vp, ctypes.POINTER(Shares), vp]),
            "spdz_mul_batch": (i32, [vp, ctypes.POINTER(Shares), ctypes.POINTER(Shares),
                                     ctypes.POINTER(Triple), ctypes.POINTER(Shares), vp, vp]),
            "spdz_mul_fused": (i32, [vp, ctypes.POINTER(Shares), ctypes.POINTER(Shares),
                                     ctypes.POINTER(Triple), ctypes.POINTER(Shares), vp, vp, u64p,
                                     ctypes.POINTER(Shares), vp, ctypes.POINTER(Shares), vp]),
            "spdz_linear": (i32, [vp, i32, ctypes.POINTER(Shares), u64p, u64p, ctypes.POINTER(Shares)]),
            "spdz_reduce_add": (i32, [vp, ctypes.POINTER(Shares), ctypes.POINTER(Shares)]),
            "spdz_mac_check": (i32, [vp, ctypes.POINTER(i32), u64p]),
            "spdz_deal_alpha": (i32, [u64p, i32, i32, ctypes.c_uint64, u64p]),
            "spdz_stream_probe": (i32, [i32, i32, vp, vp, i64, i64, i32, vp]),
            "spdz_deal_secret": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, vp,
                                       ctypes.POINTER(Shares), vp]),
            "spdz_deal_triple": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Triple)]),
            "spdz_matmul_triple": (i32, [vp, i64, i64, i64, ctypes.POINTER(Shares), ctypes.POINTER(Shares),
                                         ctypes.POINTER(Triple), ctypes.POINTER(Shares), vp, vp, i32]),
            "spdz_linear_layer": (i32, [vp, i64, i64, i64, ctypes.POINTER(Shares), ctypes.POINTER(Shares),
                                        ctypes.POINTER(Shares), ctypes.POINTER(Triple), ctypes.POINTER(Shares),
                                        vp, vp]),
            "spdz_linear_layer32": (i32, [vp, i64, i64, i64, ctypes.POINTER(Shares32), ctypes.POINTER(Shares32),
                                          ctypes.POINTER(Shares32), ctypes.POINTER(Triple32),
                                          ctypes.POINTER(Shares32), vp, vp]),
            "spdz_linear_layer_noalloc": (i32, [vp, i64, i64, i64, ctypes.POINTER(Shares), ctypes.POINTER(Shares),
                                                ctypes.POINTER(Shares), ctypes.POINTER(Triple),
                                                ctypes.POINTER(Shares), vp, vp]),
            "spdz_deal_matvec_triple": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, i64, i64, i64,
                                              ctypes.POINTER(Triple)]),
            "spdz_deal_matrix_triple": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, i64, i64, i64,
                                              ctypes.POINTER(Triple)]),
            "spdz_public_op": (i32, [vp, i32, ctypes.POINTER(Shares), vp, i64, ctypes.POINTER(Shares)]),
            "spdz_prog_create": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(vp), ctypes.c_char_p, i64]),
            "spdz_prog_destroy": (i32, [vp]),
            "spdz_prog_run": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(i32), u64p, ctypes.POINTER(ctypes.c_double)]),
            "spdz_prog_predeal": (i32, [vp, ctypes.c_uint64, i64]),
            "spdz_prog_set_fusion": (i32, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
            "spdz_prog_set_handoff": (i32, [vp, ctypes.c_int]),
            "spdz_prog_output": (i32, [vp, i32, ctypes.POINTER(Shares), vp]),
            "spdz_prog_node_info": (i32, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]),
            "spdz_prog_stats": (i32, [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
            "spdz_prog_error": (ctypes.c_char_p, [vp]),
            "spdz_dag_create": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int64), i64, vp, ctypes.POINTER(vp)]),
            "spdz_dag_destroy": (i32, [vp]),
            "spdz_dag_node": (i32, [vp, i64, ctypes.POINTER(Shares)]),
            "spdz_dag_triple": (i32, [vp, i64, ctypes.POINTER(Triple)]),
            "spdz_dag_opened_count": (i64, [vp]),
            "spdz_dag_deal": (i32, [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]),
            "spdz_dag_run": (i32, [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]),
            "spdz_dag_fetch_host_outputs": (i32, [vp]),
            "spdz_dag_set_launch": (i32, [vp, i32, i32]),
            "spdz_dag_autotune": (i32, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_double)]),
            "spdz_dag_set_threshold": (i32, [vp, i64]),
            "spdz_dag_set_flush": (i32, [vp, i64]),
            "spdz_dag_run_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(i64)]),
            "spdz_dag_time_transfer": (i32, [vp, i64, i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
            "spdz_dag_last_stats": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(ctypes.c_double)]),
            "spdz_dag_set_cost_model": (i32, [vp, vp, ctypes.c_double, ctypes.c_double]),
            "spdz_dag_time_level": (i32, [vp, i32, i64, i64, i32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
            "spdz_mlp_forward": (i32, [vp, vp, vp, i64, vp, vp]),
            "spdz_mlp_backward": (i32, [vp, vp, vp, vp, vp, i64, vp]),
            "spdz_mlp_adam": (i32, [vp, vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float]),
            "spdz_mlp_train": (i32, [vp, vp, vp, vp, i64, i32, i32, ctypes.c_float, ctypes.c_uint64, vp]),
            "spdz_timing_enable": (i32, [vp, i32]),
            "spdz_timing_get": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(i64)]),
            "spdz_copy_probe": (i32, [vp, vp, i64, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().spdz_status_str(int(s)).decode()


def _check(s: int, where: str) -> int:
    if s < 0:
        raise SpdzError(s, where)
    return s


def n_limbs(p: int) -> int:
    return 1 if p < (1 << 64) else 2


def limbs(v: int, L: int):
    return (ctypes.c_uint64 * L)(*[(v >> (64 * l)) & ((1 << 64) - 1) for l in range(L)])


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
@dataclass
class ShareTensor:
    """Values and MAC shares of a batch, device tensors [n][L][W] (canonical layout)."""
    val: torch.Tensor
    mac: torch.Tensor

    @staticmethod
    def empty(n: int, L: int, W: int, device="cuda") -> "ShareTensor":
        return ShareTensor(torch.empty((n, L, W), dtype=torch.int64, device=device),
                           torch.empty((n, L, W), dtype=torch.int64, device=device))

    @property
    def width(self) -> int:
        return self.val.shape[-1]

    def desc(self) -> Shares:
        v, m = self.val, self.mac
        assert v.is_cuda and m.is_cuda and v.dtype == torch.int64 and v.shape == m.shape
        if v.numel() == 0:
            return Shares(None, None, v.shape[2], 0, 0)
        assert v.stride() == m.stride() and v.stride(2) == 1
        return Shares(v.data_ptr(), m.data_ptr(), v.shape[2], v.stride(0), v.stride(1))


@dataclass
class TripleTensor:
    a: ShareTensor
    b: ShareTensor
    c: ShareTensor

    @staticmethod
    def empty(n, L, W, device="cuda") -> "TripleTensor":
        return TripleTensor(*(ShareTensor.empty(n, L, W, device) for _ in range(3)))

    @staticmethod
    def empty_layer(n, dout, din, tile_rows, device="cuda") -> "TripleTensor":
        """Matrix-vector triples of a linear layer: A [dout*din], B [n_tiles*din], C [dout] (one limb)."""
        n_tiles = -(-dout // tile_rows)
        return TripleTensor(ShareTensor.empty(n, 1, dout * din, device), ShareTensor.empty(n, 1, n_tiles * din, device),
                            ShareTensor.empty(n, 1, dout, device))

    @staticmethod
    def empty_matrix(n, M, K, N, device="cuda") -> "TripleTensor":
        """A [M x K], B [K x N], C [M x N] (single-limb field)."""
        return TripleTensor(ShareTensor.empty(n, 1, M * K, device), ShareTensor.empty(n, 1, K * N, device),
                            ShareTensor.empty(n, 1, M * N, device))

    def desc(self) -> Triple:
        return Triple(self.a.desc(), self.b.desc(), self.c.desc())


@dataclass
class ShareTensor32:
    """Values and MAC shares of a batch over 2^32 - 5 packed one residue per 32-bit word:
    device int32 tensors [n][W] holding the raw words (spdz_shares32)."""
    val: torch.Tensor
    mac: torch.Tensor

    @staticmethod
    def empty(n: int, W: int, device="cuda") -> "ShareTensor32":
        return ShareTensor32(torch.empty((n, W), dtype=torch.int32, device=device),
                             torch.empty((n, W), dtype=torch.int32, device=device))

    @property
    def width(self) -> int:
        return self.val.shape[-1]

    def desc(self) -> Shares32:
        v, m = self.val, self.mac
        assert v.is_cuda and m.is_cuda and v.dtype == torch.int32 and v.shape == m.shape and v.dim() == 2
        if v.numel() == 0:
            return Shares32(None, None, v.shape[1], 0)
        assert v.stride() == m.stride() and v.stride(1) == 1
        return Shares32(v.data_ptr(), m.data_ptr(), v.shape[1], v.stride(0))


@dataclass
class TripleTensor32:
    a: ShareTensor32
    b: ShareTensor32
    c: ShareTensor32

    @staticmethod
    def empty_layer(n, dout, din, tile_rows, device="cuda") -> "TripleTensor32":
        """Matrix-vector triples of a linear layer, packed: A [dout*din], B [n_tiles*din], C [dout]."""
        n_tiles = -(-dout // tile_rows)
        return TripleTensor32(ShareTensor32.empty(n, dout * din, device), ShareTensor32.empty(n, n_tiles * din, device),
                              ShareTensor32.empty(n, dout, device))

    def desc(self) -> Triple32:
        return Triple32(self.a.desc(), self.b.desc(), self.c.desc())


def spdz_copy_probe(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """Plain device copy of src into dst (int64 tensors of equal size)."""
    assert dst.numel() == src.numel() and dst.is_contiguous() and src.is_contiguous()
    st = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib().spdz_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                 src.numel(), ctypes.c_void_p(st)), "spdz_copy_probe")


def spdz_stream_probe(reads: int, writes: int, inp: Optional[torch.Tensor], out: torch.Tensor, stride: int,
                      words: int, blocks_per_cu: int = 0, stream=None):
    """Memory-pattern probe: `reads` streams read from inp and `writes` written to out (int64 tensors,
    stream k at word k * stride)."""
    st = (stream or torch.cuda.current_stream()).cuda_stream
    if inp is not None:
        assert inp.numel() >= (max(reads, 1) - 1) * stride + words
    assert out.numel() >= (max(writes, 1) - 1) * stride + words
    _check(lib().spdz_stream_probe(reads, writes, _ptr(inp), ctypes.c_void_p(out.data_ptr()), stride, words,
                                   blocks_per_cu, ctypes.c_void_p(st)), "spdz_stream_probe")


def deal_alpha(p: int, n: int, seed: int) -> list:
    """alpha_i of the fake-preprocessing dealer, as Python ints."""
    L = n_limbs(p)
    out = (ctypes.c_uint64 * (n * L))()
    _check(lib().spdz_deal_alpha(limbs(p, L), L, n, ctypes.c_uint64(seed), out), "spdz_deal_alpha")
    return [sum(int(out[i * L + l]) << (64 * l) for l in range(L)) for i in range(n)]


class Context:
    """A libspdz context (spdz_ctx) for n parties over p, on a torch stream."""

    def __init__(self, n: int, p: int, alpha_shares: Sequence[int], check_seed: int,
                 stream: Optional[torch.cuda.Stream] = None):
        self.n, self.p, self.L = n, p, n_limbs(p)
        self.alpha = list(alpha_shares)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        al = (ctypes.c_uint64 * (n * self.L))()
        for i, a in enumerate(self.alpha):
            for l in range(self.L):
                al[i * self.L + l] = (a >> (64 * l)) & ((1 << 64) - 1)
        h = ctypes.c_void_p()
        _check(lib().spdz_ctx_create(ctypes.byref(h), n, limbs(p, self.L), self.L, al,
                                     ctypes.c_uint64(check_seed),
                                     ctypes.c_void_p(self.stream.cuda_stream)), "spdz_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().spdz_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers --------------------------------------------------------------
    def new_shares(self, W: int) -> ShareTensor:
        return ShareTensor.empty(self.n, self.L, W)

    def new_public(self, W: int) -> torch.Tensor:
        return torch.empty((self.L, W), dtype=torch.int64, device="cuda")

    def opened_count(self) -> int:
        return int(lib().spdz_opened_count(self._h))

    def set_validation(self, enable: bool = True):
        """Check every input of the online-phase calls for non-canonical words (SPDZ_E_INVAL)."""
        _check(lib().spdz_ctx_set_validation(self._h, int(bool(enable))), "spdz_ctx_set_validation")

    # -- online phase ----------------------------------------------------------
    def spdz_open(self, x: ShareTensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_public(x.width) if out is None else out
        d = x.desc()
        _check(lib().spdz_open(self._h, ctypes.byref(d), _ptr(out)), "spdz_open")
        return out

    def spdz_mul_batch(self, x: ShareTensor, y: ShareTensor, t: TripleTensor, z: ShareTensor,
                       d_pub: Optional[torch.Tensor] = None, e_pub: Optional[torch.Tensor] = None):
        dx, dy, dt, dz = x.desc(), y.desc(), t.desc(), z.desc()
        _check(lib().spdz_mul_batch(self._h, ctypes.byref(dx), ctypes.byref(dy), ctypes.byref(dt),
                                    ctypes.byref(dz), _ptr(d_pub), _ptr(e_pub)), "spdz_mul_batch")
        return z

    def bind_mul_batch(self, x: ShareTensor, y: ShareTensor, t: TripleTensor, z: ShareTensor,
                       d_pub: Optional[torch.Tensor] = None, e_pub: Optional[torch.Tensor] = None):
        """spdz_mul_batch with its arguments marshalled once (see bind_mul_fused)."""
        descs = (x.desc(), y.desc(), t.desc(), z.desc())
        args = (self._h, *(ctypes.byref(d) for d in descs), _ptr(d_pub), _ptr(e_pub))
        fn = lib().spdz_mul_batch

        def call():
            st = fn(*args)
            if st != SPDZ_OK:
                raise SpdzError(st, "spdz_mul_batch")
        call._keep = (descs, (x, y, t, z, d_pub, e_pub))
        return call

    def _mul_fused_args(self, x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub):
        dx, dy, dt, dz = x.desc(), y.desc(), t.desc(), z.desc()
        lin_arr = None
        if lin is not None:
            lin_arr = (ctypes.c_uint64 * (4 * self.L))()
            for k, c in enumerate(lin):
                for l in range(self.L):
                    lin_arr[k * self.L + l] = (c >> (64 * l)) & ((1 << 64) - 1)
        dw = w.desc() if w is not None else None
        ds = s.desc() if s is not None else None
        return (self._h, ctypes.byref(dx), ctypes.byref(dy), ctypes.byref(dt), ctypes.byref(dz), _ptr(d_pub),
                _ptr(e_pub), lin_arr, ctypes.byref(dw) if dw is not None else None, _ptr(w_pub),
                ctypes.byref(ds) if ds is not None else None, _ptr(s_pub)), (dx, dy, dt, dz, dw, ds, lin_arr)

    def spdz_mul_fused(self, x, y, t, z, d_pub=None, e_pub=None, lin: Optional[Sequence[int]] = None,
                       w: Optional[ShareTensor] = None, w_pub: Optional[torch.Tensor] = None,
                       s: Optional[ShareTensor] = None, s_pub: Optional[torch.Tensor] = None):
        args, _keep = self._mul_fused_args(x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub)
        _check(lib().spdz_mul_fused(*args), "spdz_mul_fused")

    def bind_mul_fused(self, x, y, t, z, d_pub=None, e_pub=None, lin: Optional[Sequence[int]] = None,
                       w: Optional[ShareTensor] = None, w_pub: Optional[torch.Tensor] = None,
                       s: Optional[ShareTensor] = None, s_pub: Optional[torch.Tensor] = None):
        """spdz_mul_fused with its arguments marshalled once: returns a call without arguments
        that enqueues the same operation (the tensors must stay alive and in place)."""
        args, keep = self._mul_fused_args(x, y, t, z, d_pub, e_pub, lin, w, w_pub, s, s_pub)
        fn = lib().spdz_mul_fused
        tensors = (x, y, t, z, d_pub, e_pub, w, w_pub, s, s_pub)

        def call():
            st = fn(*args)
            if st != SPDZ_OK:
                raise SpdzError(st, "spdz_mul_fused")
        call._keep = (keep, tensors)
        return call

    def spdz_linear(self, terms: Sequence[ShareTensor], coeffs: Sequence[int], c0: int = 0,
                    out: Optional[ShareTensor] = None) -> ShareTensor:
        k = len(terms)
        out = self.new_shares(terms[0].width) if out is None else out
        arr = (Shares * k)(*[t.desc() for t in terms])
        cf = (ctypes.c_uint64 * (k * self.L))()
        for i, c in enumerate(coeffs):
            for l in range(self.L):
                cf[i * self.L + l] = (c >> (64 * l)) & ((1 << 64) - 1)
        do = out.desc()
        _check(lib().spdz_linear(self._h, k, arr, cf, limbs(c0, self.L), ctypes.byref(do)),
               "spdz_linear")
        return out

    def spdz_reduce_add(self, x: ShareTensor, out: Optional[ShareTensor] = None) -> ShareTensor:
        out = self.new_shares(1) if out is None else out
        dx, do = x.desc(), out.desc()
        _check(lib().spdz_reduce_add(self._h, ctypes.byref(dx), ctypes.byref(do)), "spdz_reduce_add")
        return out

    def spdz_matmul_triple(self, M: int, K: int, N: int, X: ShareTensor, Y: ShareTensor,
                           T: TripleTensor, Z: ShareTensor, E_pub: Optional[torch.Tensor] = None,
                           F_pub: Optional[torch.Tensor] = None, variant: int = -1):
        """Z = X Y with a matrix triple; matrices are [n][1][rows*cols] row-major."""
        dx, dy, dt, dz = X.desc(), Y.desc(), T.desc(), Z.desc()
        _check(lib().spdz_matmul_triple(self._h, M, K, N, ctypes.byref(dx), ctypes.byref(dy),
                                        ctypes.byref(dt), ctypes.byref(dz), _ptr(E_pub), _ptr(F_pub),
                                        variant), "spdz_matmul_triple")
        return Z

    def spdz_linear_layer(self, dout: int, din: int, tile_rows: int, W: ShareTensor, x: ShareTensor,
                          b: ShareTensor, T: TripleTensor, y: Optional[ShareTensor] = None,
                          D_pub: Optional[torch.Tensor] = None, E_pub: Optional[torch.Tensor] = None) -> ShareTensor:
        """y = W x + b with one matrix-vector triple per tile of tile_rows rows (W row-major
        [n][1][dout*din], x [n][1][din], b and y [n][1][dout], T.b [n][1][n_tiles*din])."""
        y = self.new_shares(dout) if y is None else y
        dW, dx, db, dt, dy = W.desc(), x.desc(), b.desc(), T.desc(), y.desc()
        _check(lib().spdz_linear_layer(self._h, dout, din, tile_rows, ctypes.byref(dW), ctypes.byref(dx),
                                       ctypes.byref(db), ctypes.byref(dt), ctypes.byref(dy), _ptr(D_pub),
                                       _ptr(E_pub)), "spdz_linear_layer")
        return y

    def spdz_linear_layer32(self, dout: int, din: int, tile_rows: int, W: ShareTensor32, x: ShareTensor32,
                            b: ShareTensor32, T: TripleTensor32, y: Optional[ShareTensor32] = None,
                            D_pub: Optional[torch.Tensor] = None,
                            E_pub: Optional[torch.Tensor] = None) -> ShareTensor32:
        """spdz_linear_layer on residues of 2^32 - 5 packed in 32-bit words (int32 tensors [n][len];
        D_pub [dout*din] and E_pub [n_tiles*din] int32)."""
        y = ShareTensor32.empty(self.n, dout) if y is None else y
        dW, dx, db, dt, dy = W.desc(), x.desc(), b.desc(), T.desc(), y.desc()
        _check(lib().spdz_linear_layer32(self._h, dout, din, tile_rows, ctypes.byref(dW), ctypes.byref(dx),
                                         ctypes.byref(db), ctypes.byref(dt), ctypes.byref(dy), _ptr(D_pub),
                                         _ptr(E_pub)), "spdz_linear_layer32")
        return y

    def spdz_linear_layer_noalloc(self, dout: int, din: int, tile_rows: int, W: ShareTensor, x: ShareTensor,
                                  b: ShareTensor, T: TripleTensor, y: ShareTensor,
                                  D_pub: Optional[torch.Tensor] = None,
                                  E_pub: Optional[torch.Tensor] = None) -> ShareTensor:
        """spdz_linear_layer with no allocation: y must be given; without E_pub the opened E_t use
        the library's fixed per-GPU scratch (n_tiles * din <= NOALLOC_SCRATCH_WORDS)."""
        dW, dx, db, dt, dy = W.desc(), x.desc(), b.desc(), T.desc(), y.desc()
        _check(lib().spdz_linear_layer_noalloc(self._h, dout, din, tile_rows, ctypes.byref(dW), ctypes.byref(dx),
                                               ctypes.byref(db), ctypes.byref(dt), ctypes.byref(dy), _ptr(D_pub),
                                               _ptr(E_pub)), "spdz_linear_layer_noalloc")
        return y

    def spdz_mac_check(self):
        """(accepted, [sigma_i as ints])."""
        acc = ctypes.c_int(0)
        sig = (ctypes.c_uint64 * (self.n * self.L))()
        s = _check(lib().spdz_mac_check(self._h, ctypes.byref(acc), sig), "spdz_mac_check")
        sigma = [sum(int(sig[i * self.L + l]) << (64 * l) for l in range(self.L)) for i in range(self.n)]
        return bool(acc.value) and s == SPDZ_OK, sigma

    def bind_mac_check(self):
        """spdz_mac_check with its output buffers made once: returns a call without arguments that
        returns the verdict (sigma stays in the bound buffer)."""
        acc = ctypes.c_int(0)
        sig = (ctypes.c_uint64 * (self.n * self.L))()
        fn, h, pacc = lib().spdz_mac_check, self._h, ctypes.byref(acc)

        def call() -> bool:
            st = fn(h, pacc, sig)
            if st not in (SPDZ_OK, SPDZ_MAC_REJECT):
                raise SpdzError(st, "spdz_mac_check")
            return st == SPDZ_OK and bool(acc.value)
        call._keep = (acc, sig)
        return call

    # -- measurement ------------------------------------------------------------
    def spdz_timing_enable(self, enable: bool = True):
        _check(lib().spdz_timing_enable(self._h, int(enable)), "spdz_timing_enable")

    def spdz_timing_get(self, kernel: str):
        """(total ms, launches) of a kernel since timing was enabled."""
        ms = ctypes.c_double(0)
        cnt = ctypes.c_int64(0)
        _check(lib().spdz_timing_get(self._h, kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
               "spdz_timing_get")
        return ms.value, cnt.value

    # -- fake preprocessing ---------------------------------------------------
    def spdz_deal_secret(self, seed: int, array_id: int, out: ShareTensor,
                         values: Optional[torch.Tensor] = None,
                         values_out: Optional[torch.Tensor] = None) -> ShareTensor:
        d = out.desc()
        _check(lib().spdz_deal_secret(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(array_id),
                                      _ptr(values), ctypes.byref(d), _ptr(values_out)),
               "spdz_deal_secret")
        return out

    def spdz_deal_matrix_triple(self, seed: int, array_id: int, M: int, K: int, N: int,
                                out: TripleTensor) -> TripleTensor:
        d = out.desc()
        _check(lib().spdz_deal_matrix_triple(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(array_id),
                                             M, K, N, ctypes.byref(d)), "spdz_deal_matrix_triple")
        return out

    def spdz_deal_matvec_triple(self, seed: int, array_id: int, dout: int, din: int, tile_rows: int,
                                out: TripleTensor) -> TripleTensor:
        d = out.desc()
        _check(lib().spdz_deal_matvec_triple(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(array_id),
                                             dout, din, tile_rows, ctypes.byref(d)), "spdz_deal_matvec_triple")
        return out

    def spdz_deal_triple(self, seed: int, array_id: int, out: TripleTensor) -> TripleTensor:
        d = out.desc()
        _check(lib().spdz_deal_triple(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(array_id),
                                      ctypes.byref(d)), "spdz_deal_triple")
        return out


# ---------------------------------------------------------------------------
# DAG execution
# ---------------------------------------------------------------------------
MODE_PER_OP, MODE_PER_LEVEL, MODE_GRAPH = 0, 1, 2
POLICY_STATIC, POLICY_LEARNED, POLICY_ALL_GPU, POLICY_ALL_CPU = 0, 1, 2, 3

DAG_OP_DTYPE = None


def dag_op_dtype():
    import numpy as np
    global DAG_OP_DTYPE
    if DAG_OP_DTYPE is None:
        DAG_OP_DTYPE = np.dtype([("kind", np.int32), ("level", np.int32), ("width", np.int64),
                                 ("src1", np.int64), ("off1", np.int64), ("src2", np.int64),
                                 ("off2", np.int64), ("konst", np.uint64)])
    return DAG_OP_DTYPE


SPDZ_PUB_ADD, SPDZ_PUB_MUL, SPDZ_PUB_SHARE, SPDZ_PUB_SUB = 0, 1, 2, 3


def public_op(ctx: "Context", mode: int, x: Optional[ShareTensor], v: torch.Tensor, out: ShareTensor) -> ShareTensor:
    """out = x + v, x * v (element-wise) or share(v); v is a [L][W] or [L][1] device tensor."""
    dx = x.desc() if x is not None else None
    do = out.desc()
    _check(lib().spdz_public_op(ctx._h, mode, ctypes.byref(dx) if dx is not None else None, _ptr(v), v.shape[-1],
                                ctypes.byref(do)), "spdz_public_op")
    return out


class ProgramError(Exception):
    pass


class Program:
    """A control-flow program (text format of workloads.programs) on a context."""

    def __init__(self, ctx: "Context", text: str, fuse: bool = True, handoff: bool = True):
        self.ctx = ctx
        h = ctypes.c_void_p()
        err = ctypes.create_string_buffer(512)
        st = lib().spdz_prog_create(ctx._h, text.encode(), ctypes.byref(h), err, 512)
        if st != SPDZ_OK:
            raise ProgramError(f"spdz_prog_create: {status_str(st)}: {err.value.decode()}")
        self._h = h
        self.n_groups = self.set_fusion(fuse)
        self.set_handoff(handoff)

    def set_fusion(self, enable: bool) -> int:
        """Fused element-wise runs on or off; returns the number of fused runs of the program."""
        ng = ctypes.c_int(0)
        _check(lib().spdz_prog_set_fusion(self._h, int(bool(enable)), ctypes.byref(ng)), "spdz_prog_set_fusion")
        return ng.value

    def set_handoff(self, enable: bool):
        """Phi buffer hand-off on (a loop-carried value moves) or off (every phi copies)."""
        _check(lib().spdz_prog_set_handoff(self._h, int(bool(enable))), "spdz_prog_set_handoff")

    def close(self):
        if getattr(self, "_h", None):
            lib().spdz_prog_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, seed: int):
        """(accepted, [sigma_i as ints], wall_ms)."""
        acc = ctypes.c_int(0)
        n, L = self.ctx.n, self.ctx.L
        sig = (ctypes.c_uint64 * (n * L))()
        ms = ctypes.c_double(0)
        st = lib().spdz_prog_run(self._h, ctypes.c_uint64(seed), ctypes.byref(acc), sig, ctypes.byref(ms))
        if st not in (SPDZ_OK, SPDZ_MAC_REJECT):
            msg = lib().spdz_prog_error(self._h)
            raise SpdzError(st, f"spdz_prog_run: {msg.decode() if msg else ''}")
        sigma = [sum(int(sig[i * L + l]) << (64 * l) for l in range(L)) for i in range(n)]
        return bool(acc.value) and st == SPDZ_OK, sigma, ms.value

    def predeal(self, seed: int, executions: int):
        """Deal the triples of the first `executions` executions of every product / layer node ahead."""
        _check(lib().spdz_prog_predeal(self._h, ctypes.c_uint64(seed), executions), "spdz_prog_predeal")

    def info(self, node: int):
        sec, w = ctypes.c_int(0), ctypes.c_int64(0)
        _check(lib().spdz_prog_node_info(self._h, node, ctypes.byref(sec), ctypes.byref(w)), "spdz_prog_node_info")
        return bool(sec.value), int(w.value)

    def output(self, node: int):
        """ShareTensor for a secret output, a [L][width] device tensor for a public one."""
        secret, w = self.info(node)
        if secret:
            out = self.ctx.new_shares(w)
            d = out.desc()
            _check(lib().spdz_prog_output(self._h, node, ctypes.byref(d), None), "spdz_prog_output")
        else:
            out = self.ctx.new_public(w)
            _check(lib().spdz_prog_output(self._h, node, None, _ptr(out)), "spdz_prog_output")
        return out

    def stats(self):
        v = [ctypes.c_int64(0) for _ in range(4)]
        _check(lib().spdz_prog_stats(self._h, *[ctypes.byref(x) for x in v]), "spdz_prog_stats")
        return dict(zip(("block_entries", "launches", "host_syncs", "opened"), (int(x.value) for x in v)))


class Dag:
    """A spdz_dag built from an op table (numpy array of dag_op_dtype())."""

    def __init__(self, ctx: Context, input_widths, ops):
        import numpy as np
        self.ctx = ctx
        ops = np.ascontiguousarray(ops, dtype=dag_op_dtype())
        self._ops = ops
        iw = (ctypes.c_int64 * len(input_widths))(*input_widths)
        h = ctypes.c_void_p()
        _check(lib().spdz_dag_create(ctx._h, len(input_widths), iw, len(ops), ops.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(h)), "spdz_dag_create")
        self._h = h
        self.n_inputs = len(input_widths)
        self.input_widths = list(input_widths)

    def close(self):
        if getattr(self, "_h", None):
            lib().spdz_dag_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def opened_count(self) -> int:
        return int(lib().spdz_dag_opened_count(self._h))

    def deal(self, seed: int, input_array0: int, triple_array0: int):
        _check(lib().spdz_dag_deal(self._h, ctypes.c_uint64(seed), ctypes.c_uint64(input_array0),
                                   ctypes.c_uint64(triple_array0)), "spdz_dag_deal")

    def run(self, mode: int = MODE_PER_LEVEL, policy: int = POLICY_ALL_GPU) -> float:
        ms = ctypes.c_double(0)
        _check(lib().spdz_dag_run(self._h, mode, policy, ctypes.byref(ms)), "spdz_dag_run")
        return ms.value

    def fetch_host_outputs(self):
        _check(lib().spdz_dag_fetch_host_outputs(self._h), "spdz_dag_fetch_host_outputs")

    def node(self, k: int) -> ShareTensor:
        """Copy of node k's shares into fresh tensors [n][1][width]."""
        d = Shares()
        _check(lib().spdz_dag_node(self._h, k, ctypes.byref(d)), "spdz_dag_node")
        n = self.ctx.n
        out = ShareTensor.empty(n, 1, d.len)
        st = ctypes.c_void_p(self.ctx.stream.cuda_stream)
        _check(lib().spdz_copy_probe(ctypes.c_void_p(out.val.data_ptr()), ctypes.c_void_p(d.val), n * d.len, st),
               "spdz_copy_probe")
        _check(lib().spdz_copy_probe(ctypes.c_void_p(out.mac.data_ptr()), ctypes.c_void_p(d.mac), n * d.len, st),
               "spdz_copy_probe")
        return out

    def node_arena(self):
        """Copies of the whole value and MAC arenas (int64 device tensors of n * sum(widths) words):
        node k's [n][width] shares start at n * (sum of the widths of nodes before k)."""
        d = Shares()
        _check(lib().spdz_dag_node(self._h, 0, ctypes.byref(d)), "spdz_dag_node")
        widths = [int(w) for w in self.input_widths] + [int(w) for w in self._ops["width"]]
        words = self.ctx.n * sum(widths)
        st = ctypes.c_void_p(self.ctx.stream.cuda_stream)
        val = torch.empty(words, dtype=torch.int64, device="cuda")
        mac = torch.empty(words, dtype=torch.int64, device="cuda")
        _check(lib().spdz_copy_probe(ctypes.c_void_p(val.data_ptr()), ctypes.c_void_p(d.val), words, st),
               "spdz_copy_probe")
        _check(lib().spdz_copy_probe(ctypes.c_void_p(mac.data_ptr()), ctypes.c_void_p(d.mac), words, st),
               "spdz_copy_probe")
        return val, mac

    def set_launch(self, tile: int, blocks_per_cu: int):
        _check(lib().spdz_dag_set_launch(self._h, tile, blocks_per_cu), "spdz_dag_set_launch")

    def autotune(self, max_levels: int = 20):
        t, b = ctypes.c_int(0), ctypes.c_int(0)
        ms = ctypes.c_double(0)
        _check(lib().spdz_dag_autotune(self._h, max_levels, ctypes.byref(t), ctypes.byref(b), ctypes.byref(ms)),
               "spdz_dag_autotune")
        return t.value, b.value, ms.value

    def set_threshold(self, thr: int):
        _check(lib().spdz_dag_set_threshold(self._h, thr), "spdz_dag_set_threshold")

    def set_flush(self, flush_elems: int):
        """Static batch flush point of the scheduler, in elements (0: one launch per level)."""
        _check(lib().spdz_dag_set_flush(self._h, flush_elems), "spdz_dag_set_flush")

    def run_info(self):
        v = [ctypes.c_int64(0) for _ in range(4)]
        _check(lib().spdz_dag_run_info(self._h, *(ctypes.byref(x) for x in v)), "spdz_dag_run_info")
        return dict(zip(("launches", "early_flushes", "transfers", "transfer_bytes"), (x.value for x in v)))

    def last_stats(self):
        g, c, cp = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        pm = ctypes.c_double(0)
        _check(lib().spdz_dag_last_stats(self._h, ctypes.byref(g), ctypes.byref(c), ctypes.byref(cp),
                                         ctypes.byref(pm)), "spdz_dag_last_stats")
        return dict(gpu_ops=g.value, cpu_ops=c.value, copies=cp.value, predict_ms=pm.value)

    def set_cost_model(self, weights, ns_per_byte: float, ns_per_copy: float):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.float32)
        assert w.size == MLP_NPARAM
        _check(lib().spdz_dag_set_cost_model(self._h, w.ctypes.data_as(ctypes.c_void_p), ns_per_byte, ns_per_copy),
               "spdz_dag_set_cost_model")


def dag_time_transfer(ctx: Context, words: int, reps: int = 5):
    """(device-to-host ns, host-to-device ns) of one hybrid-run transfer of `words` 64-bit words."""
    d, h = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().spdz_dag_time_transfer(ctx._h, words, reps, ctypes.byref(d), ctypes.byref(h)),
           "spdz_dag_time_transfer")
    return d.value, h.value


def dag_time_level(ctx: Context, kind: int, width: int, q: int, reps: int = 3):
    """(gpu ns per op, cpu ns per op, q used) for one level of q ops."""
    g, c = ctypes.c_double(0), ctypes.c_double(0)
    qu = ctypes.c_int64(0)
    _check(lib().spdz_dag_time_level(ctx._h, kind, width, q, reps, ctypes.byref(g), ctypes.byref(c),
                                     ctypes.byref(qu)), "spdz_dag_time_level")
    return g.value, c.value, qu.value


# ---------------------------------------------------------------------------
# cost-model MLP (device tensors float32)
# ---------------------------------------------------------------------------
MLP_IN, MLP_HID, MLP_OUT, MLP_NPARAM = 7, 64, 2, 8962


def _st(stream):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def mlp_forward(W: torch.Tensor, X: torch.Tensor, acts: bool = False, stream=None):
    B = X.shape[0]
    Y = torch.empty((B, MLP_OUT), dtype=torch.float32, device="cuda")
    A = torch.empty((3, B, MLP_HID), dtype=torch.float32, device="cuda") if acts else None
    _check(lib().spdz_mlp_forward(_st(stream), _ptr(W), _ptr(X), B, _ptr(Y), _ptr(A)), "spdz_mlp_forward")
    return (Y, A) if acts else Y


def mlp_backward(W, X, A, dY, stream=None):
    dW = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    _check(lib().spdz_mlp_backward(_st(stream), _ptr(W), _ptr(X), _ptr(A), _ptr(dY), X.shape[0], _ptr(dW)),
           "spdz_mlp_backward")
    return dW


def mlp_adam(W, dW, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _check(lib().spdz_mlp_adam(_st(stream), _ptr(W), _ptr(dW), _ptr(m), _ptr(v), t, lr, b1, b2, eps), "spdz_mlp_adam")


def mlp_train(W, X, T, epochs: int, batch: int, lr: float, seed: int, stream=None):
    import numpy as np
    loss = np.zeros(epochs, dtype=np.float32)
    _check(lib().spdz_mlp_train(_st(stream), _ptr(W), _ptr(X), _ptr(T), X.shape[0], epochs, batch, lr,
                                ctypes.c_uint64(seed), loss.ctypes.data_as(ctypes.c_void_p)), "spdz_mlp_train")
    return loss
