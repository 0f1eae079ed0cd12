"""Python binding of libzk.so (include/zk.h): argument marshalling only.

Device buffers are torch tensors on a ROCm device holding raw 32-bit words
(dtype torch.int32, reinterpreted as unsigned by the library):

* field elements: shape (n, 8), canonical little-endian limbs;
* affine G1 points: shape (n, 16), x then y; (0, 0) is the point at infinity.

Every call enqueues on torch's current stream of the tensors' device.  There
is no fallback: if libzk.so is missing the import of this module raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzk.so")

ZK_OK, ZK_EINVAL, ZK_ENOMEM, ZK_EDEVICE, ZK_EBUDGET, ZK_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MAX_LOG_NTT = 28

EXPORTS = ("zk_last_error", "zk_ntt", "zk_intt", "zk_coset_ntt", "zk_msm", "zk_srs_setup", "zk_srs_create",
           "zk_srs_destroy", "zk_srs_size", "zk_msm_srs", "zk_msm_batch", "zk_fold", "zk_profile_enable",
           "zk_profile_read", "zk_msm_srs_workspace_bytes", "zk_ntt_workspace_bytes", "zk_release_cached_memory",
           "zk_msm_srs_ex", "zk_profile_only", "zk_commit_job", "zk_set_validate", "zk_kzg_open",
           "zk_kzg_open_batch", "zk_quotient_mul",
           "zk_srs_lagrange_setup", "zk_transcript_challenge", "zk_acc_fold",
           "zk_srs_g2_setup", "zk_srs_g2_create", "zk_srs_g2_destroy", "zk_srs_g2_size", "zk_msm_g2_srs",
           "zk_srs_set_table_policy", "zk_srs_set_tiny_max", "zk_srs_window_bits", "zk_set_scratch_budget", "zk_scratch_held", "zk_msm_srs_noalloc",
           "zk_quotient_polyiop", "zk_calibrate_mad_rate", "zk_set_schedule", "zk_get_schedule")


class ZkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("zk error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libzk.so not built (run python -m paper_2507_07031_amd.build): %s" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "zk_last_error": ([], ctypes.c_char_p),
        "zk_ntt": ([P, P, U32, P], I),
        "zk_intt": ([P, P, U32, P], I),
        "zk_coset_ntt": ([P, U32, U32, P, P, P], I),
        "zk_msm": ([P, P, U64, P, P], I),
        "zk_srs_setup": ([P, U64, P, P], I),
        "zk_srs_lagrange_setup": ([P, U32, P, P], I),
        "zk_srs_create": ([P, U64, ctypes.POINTER(ctypes.c_void_p), P], I),
        "zk_srs_destroy": ([P], I),
        "zk_srs_size": ([P], U64),
        "zk_msm_srs": ([P, P, U64, P, P], I),
        "zk_msm_srs_ex": ([P, P, U64, P, P, P], I),
        "zk_msm_srs_noalloc": ([P, P, U64, P, P], I),
        "zk_profile_only": ([ctypes.c_char_p], I),
        "zk_set_validate": ([I], I),
        "zk_commit_job": ([P, P, I, I, P, P, P, P, P], I),
        "zk_msm_batch": ([P, P, P, U32, P, P], I),
        "zk_kzg_open": ([P, P, U64, P, P, P, P, P], I),
        "zk_quotient_mul": ([P, P, P, P, U32, U32, P, P, P, P], I),
        "zk_quotient_polyiop": ([P, P, U32, U32, P, U32, U32, P, P, P, P], I),
        "zk_calibrate_mad_rate": ([U32, U32, ctypes.POINTER(ctypes.c_double), P], I),
        "zk_set_schedule": ([P], I),
        "zk_get_schedule": ([P], I),
        "zk_transcript_challenge": ([P, U64, P, P], I),
        "zk_srs_g2_setup": ([P, U64, P, P], I),
        "zk_srs_g2_create": ([P, U64, ctypes.POINTER(ctypes.c_void_p), P], I),
        "zk_srs_g2_destroy": ([P], I),
        "zk_srs_g2_size": ([P], U64),
        "zk_msm_g2_srs": ([P, P, U64, P, P], I),
        "zk_srs_set_table_policy": ([P, U64, U64], I),
        "zk_srs_set_tiny_max": ([P, U64], I),
        "zk_srs_window_bits": ([P, U64], U32),
        "zk_acc_fold": ([U32, P, P, U32, P, P, P, U64, P, P, U64, P, P, P, P, P, P, P, P, P], I),
        "zk_kzg_open_batch": ([P, P, U32, U64, P, P, P, P, P, P], I),
        "zk_fold": ([P, P, U32, U32, P, P], I),
        "zk_profile_enable": ([I], I),
        "zk_release_cached_memory": ([], I),
        "zk_set_scratch_budget": ([U64], I),
        "zk_scratch_held": ([], U64),
        "zk_msm_srs_workspace_bytes": ([P, U64], U64),
        "zk_ntt_workspace_bytes": ([U32], U64),
        "zk_profile_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U64), I], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(code):
    if code != ZK_OK:
        raise ZkError(code, lib.zk_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_words(t, width, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != torch.int32 or t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
        raise TypeError("%s must be a contiguous int32 tensor of shape (n, %d)" % (name, width))
    return t


def _host_fr(words):
    a = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).reshape(8))
    return a, a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- transfers

def to_device(arr, device="cuda"):
    """numpy uint32 array -> int32 device tensor with the same bits."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host(t):
    """int32 device tensor -> numpy uint32 array with the same bits."""
    return t.detach().cpu().numpy().view(np.uint32)


# ---------------------------------------------------------------- transforms

def ntt(x, out=None, log_n=None):
    x = _dev_words(x, 8, "x")
    n = x.shape[0]
    L = int(log_n if log_n is not None else n.bit_length() - 1)
    if (1 << L) != n:
        raise ValueError("length must be a power of two")
    out = out if out is not None else _torch().empty_like(x)
    _check(lib.zk_ntt(_ptr(x), _ptr(out), L, _stream(x)))
    return out


def intt(x, out=None):
    x = _dev_words(x, 8, "x")
    n = x.shape[0]
    L = n.bit_length() - 1
    if (1 << L) != n:
        raise ValueError("length must be a power of two")
    out = out if out is not None else _torch().empty_like(x)
    _check(lib.zk_intt(_ptr(x), _ptr(out), L, _stream(x)))
    return out


def coset_ntt(coeffs, log_blowup, shift=None, out=None):
    coeffs = _dev_words(coeffs, 8, "coeffs")
    n = coeffs.shape[0]
    L = n.bit_length() - 1
    if (1 << L) != n:
        raise ValueError("length must be a power of two")
    torch = _torch()
    if out is None:
        out = torch.empty((n << log_blowup, 8), dtype=torch.int32, device=coeffs.device)
    sp = None
    if shift is not None:
        sa, sp = _host_fr(shift)
    _check(lib.zk_coset_ntt(_ptr(coeffs), L, int(log_blowup), sp, _ptr(out), _stream(coeffs)))
    return out


# ---------------------------------------------------------------- commitments

def commit_job(srs, evals, log_blowup=2, shift=None, coeffs=None, com=None, coset=None):
    """iNTT -> commitment against the SRS -> coset evaluations, overlapped by
    the library.  Returns (coeffs, com, coset)."""
    evals = _dev_words(evals, 8, "evals")
    n = evals.shape[0]
    L = n.bit_length() - 1
    if (1 << L) != n:
        raise ValueError("length must be a power of two")
    torch = _torch()
    if coeffs is None:
        coeffs = torch.empty_like(evals)
    if com is None:
        com = torch.empty((1, 16), dtype=torch.int32, device=evals.device)
    if coset is None:
        coset = torch.empty((n << log_blowup, 8), dtype=torch.int32, device=evals.device)
    sp = None
    if shift is not None:
        sa, sp = _host_fr(shift)
    _check(lib.zk_commit_job(srs.handle, _ptr(evals), L, int(log_blowup), sp, _ptr(coeffs), _ptr(com), _ptr(coset),
                             _stream(evals)))
    return coeffs, com, coset


def msm(bases, scalars, n=None, out=None):
    bases = _dev_words(bases, 16, "bases")
    scalars = _dev_words(scalars, 8, "scalars")
    n = int(n if n is not None else scalars.shape[0])
    if n > bases.shape[0] or n > scalars.shape[0]:
        raise ValueError("n exceeds the inputs")
    if out is None:
        out = _torch().empty((1, 16), dtype=_torch().int32, device=bases.device)
    _check(lib.zk_msm(_ptr(bases), _ptr(scalars), n, _ptr(out), _stream(bases)))
    return out


def srs_setup(tau, n, device="cuda"):
    torch = _torch()
    out = torch.empty((int(n), 16), dtype=torch.int32, device=device)
    ta, tp = _host_fr(tau)
    _check(lib.zk_srs_setup(tp, int(n), _ptr(out), _stream(out)))
    return out


def srs_lagrange_setup(tau, log_n, device="cuda"):
    """[l_j(tau)]_1 for the Lagrange basis of the 2^log_n-th roots of unity."""
    torch = _torch()
    out = torch.empty((1 << int(log_n), 16), dtype=torch.int32, device=device)
    ta, tp = _host_fr(tau)
    _check(lib.zk_srs_lagrange_setup(tp, int(log_n), _ptr(out), _stream(out)))
    return out


class SRS:
    """A prepared SRS (zk_srs handle) built from device points (n, 16)."""

    def __init__(self, points):
        points = _dev_words(points, 16, "points")
        h = ctypes.c_void_p()
        _check(lib.zk_srs_create(_ptr(points), points.shape[0], ctypes.byref(h), _stream(points)))
        self.handle = h
        self.device = points.device
        self.n = int(lib.zk_srs_size(h))

    def close(self):
        if self.handle:
            _check(lib.zk_srs_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def srs_set_table_policy(srs, small_max, large_min):
    """n < small_max: 12-bit-window table (first 2^16 points); n >= large_min:
    20-bit (if built); 16-bit otherwise."""
    _check(lib.zk_srs_set_table_policy(srs.handle, int(small_max), int(large_min)))


def srs_set_tiny_max(srs, tiny_max):
    """Commitments of 0 < n <= tiny_max points run on the small-multiples
    table (default 4096; 0 turns it off)."""
    _check(lib.zk_srs_set_tiny_max(srs.handle, int(tiny_max)))


SCHEDULE_FIELDS = ("acc_max_slice", "acc_blocks_per_cu", "reduce_chunk", "sort_chunk", "sort_bin_entries",
                   "ntt_tile_log", "ntt_unit_log", "ntt_overlap_tile_log")


class Schedule(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in SCHEDULE_FIELDS]


def set_schedule(values=None):
    """Launch schedule of the current device from a dict of SCHEDULE_FIELDS
    (missing or 0: built-in value); None restores every default."""
    if values is None:
        _check(lib.zk_set_schedule(None))
        return
    unknown = set(values) - set(SCHEDULE_FIELDS)
    if unknown:
        raise ValueError("unknown schedule fields: %s" % sorted(unknown))
    sch = Schedule(*[int(values.get(f, 0)) for f in SCHEDULE_FIELDS])
    _check(lib.zk_set_schedule(ctypes.byref(sch)))


def get_schedule():
    sch = Schedule()
    _check(lib.zk_get_schedule(ctypes.byref(sch)))
    return {f: int(getattr(sch, f)) for f in SCHEDULE_FIELDS}


def srs_window_bits(srs, n):
    return int(lib.zk_srs_window_bits(srs.handle, int(n)))


def msm_srs(srs, scalars, n=None, out=None):
    scalars = _dev_words(scalars, 8, "scalars")
    n = int(n if n is not None else scalars.shape[0])
    if n > scalars.shape[0]:
        raise ValueError("n exceeds the scalars")
    if out is None:
        out = _torch().empty((1, 16), dtype=_torch().int32, device=scalars.device)
    _check(lib.zk_msm_srs(srs.handle, _ptr(scalars), n, _ptr(out), _stream(scalars)))
    return out


def msm_srs_noalloc(srs, scalars, out, n=None):
    """msm_srs with the library's fixed scratch array (no allocation; up to
    2^18 points).  `out` is required: a (1, 16) device tensor."""
    scalars = _dev_words(scalars, 8, "scalars")
    out = _dev_words(out, 16, "out")
    n = int(n if n is not None else scalars.shape[0])
    if n > scalars.shape[0]:
        raise ValueError("n exceeds the scalars")
    _check(lib.zk_msm_srs_noalloc(srs.handle, _ptr(scalars), n, _ptr(out), _stream(scalars)))
    return out


def msm_srs_overlap(srs, scalars, accumulate_done, n=None, out=None):
    """msm_srs that records the torch.cuda.Event `accumulate_done` on the
    current stream right after the bucket-accumulation kernel."""
    scalars = _dev_words(scalars, 8, "scalars")
    n = int(n if n is not None else scalars.shape[0])
    if n > scalars.shape[0]:
        raise ValueError("n exceeds the scalars")
    if out is None:
        out = _torch().empty((1, 16), dtype=_torch().int32, device=scalars.device)
    ev = ctypes.c_void_p(accumulate_done.cuda_event)
    _check(lib.zk_msm_srs_ex(srs.handle, _ptr(scalars), n, _ptr(out), _stream(scalars), ev))
    return out


def msm_batch(srs, scalars, offsets, out=None):
    scalars = _dev_words(scalars, 8, "scalars")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    batch = off.shape[0] - 1
    if batch < 0 or int(off[-1]) > scalars.shape[0]:
        raise ValueError("offsets exceed the scalars")
    if out is None:
        out = _torch().empty((max(batch, 0), 16), dtype=_torch().int32, device=scalars.device)
    _check(lib.zk_msm_batch(srs.handle, _ptr(scalars), off.ctypes.data_as(ctypes.c_void_p), batch, _ptr(out),
                            _stream(scalars)))
    return out


def kzg_open(srs, coeffs, x, n=None, y=None, quotient=None, proof=None, want_quotient=False):
    """KZG opening of the polynomial with coefficients `coeffs` (n, 8) at the
    host Fr value x (8 words).  Returns (y, quotient or None, proof)."""
    coeffs = _dev_words(coeffs, 8, "coeffs")
    n = int(n if n is not None else coeffs.shape[0])
    if n > coeffs.shape[0]:
        raise ValueError("n exceeds the coefficients")
    torch = _torch()
    dev = coeffs.device
    if y is None:
        y = torch.empty((1, 8), dtype=torch.int32, device=dev)
    if quotient is None and want_quotient:
        quotient = torch.empty((max(n - 1, 0), 8), dtype=torch.int32, device=dev)
    if proof is None:
        proof = torch.empty((1, 16), dtype=torch.int32, device=dev)
    xa, xp = _host_fr(x)
    qp = _ptr(quotient) if quotient is not None else None
    _check(lib.zk_kzg_open(srs.handle, _ptr(coeffs), n, xp, _ptr(y), qp, _ptr(proof), _stream(coeffs)))
    return y, quotient, proof


def kzg_open_batch(srs, polys, x, gamma, ys=None, quotient=None, proof=None, want_quotient=False):
    """Batched opening of m polynomials polys (m, n, 8) at x with challenge
    gamma (host Fr values).  Returns (ys (m, 8), quotient or None, proof)."""
    torch = _torch()
    if (not isinstance(polys, torch.Tensor) or not polys.is_cuda or polys.dim() != 3 or polys.shape[2] != 8
            or polys.dtype != torch.int32 or not polys.is_contiguous()):
        raise TypeError("polys must be a contiguous int32 device tensor of shape (m, n, 8)")
    m, n = int(polys.shape[0]), int(polys.shape[1])
    dev = polys.device
    if ys is None:
        ys = torch.empty((m, 8), dtype=torch.int32, device=dev)
    if quotient is None and want_quotient:
        quotient = torch.empty((max(n - 1, 0), 8), dtype=torch.int32, device=dev)
    if proof is None:
        proof = torch.empty((1, 16), dtype=torch.int32, device=dev)
    xa, xp = _host_fr(x)
    ga, gp = _host_fr(gamma)
    qp = _ptr(quotient) if quotient is not None else None
    _check(lib.zk_kzg_open_batch(srs.handle, _ptr(polys), m, n, xp, gp, _ptr(ys), qp, _ptr(proof),
                                 _stream(polys)))
    return ys, quotient, proof


def quotient_mul(srs, a, b, c, log_blowup=1, shift=None, t=None, com=None):
    """Mul-block quotient t = (f h - g) / (X^n - 1) of witness vectors a, b, c
    (each (n, 8), n a power of two) and its commitment.  Returns (t, com)."""
    a = _dev_words(a, 8, "a")
    b = _dev_words(b, 8, "b")
    c = _dev_words(c, 8, "c")
    n = a.shape[0]
    L = n.bit_length() - 1
    if (1 << L) != n or b.shape[0] != n or c.shape[0] != n:
        raise ValueError("a, b, c must have one power-of-two length")
    torch = _torch()
    if t is None:
        t = torch.empty_like(a)
    if com is None:
        com = torch.empty((1, 16), dtype=torch.int32, device=a.device)
    sp = None
    if shift is not None:
        sa, sp = _host_fr(shift)
    _check(lib.zk_quotient_mul(srs.handle, _ptr(a), _ptr(b), _ptr(c), L, int(log_blowup), sp, _ptr(t), _ptr(com),
                               _stream(a)))
    return t, com


POLYIOP_MAX_WITNESS, POLYIOP_MAX_TERMS, POLYIOP_MAX_DEGREE = 8, 16, 4


class ConstraintTerm(ctypes.Structure):
    """zk_constraint_term: coeff (8 words), nfactors, factor[4]."""
    _fields_ = [("coeff", ctypes.c_uint32 * 8), ("nfactors", ctypes.c_uint32),
                ("factor", ctypes.c_uint32 * POLYIOP_MAX_DEGREE)]


def _terms_array(terms):
    arr = (ConstraintTerm * max(len(terms), 1))()
    for t, (c, factors) in enumerate(terms):
        c = int(c)
        for i in range(8):
            arr[t].coeff[i] = (c >> (32 * i)) & 0xFFFFFFFF
        arr[t].nfactors = len(factors)
        for i, a in enumerate(list(factors)[:POLYIOP_MAX_DEGREE]):
            arr[t].factor[i] = int(a)
    return arr


def quotient_polyiop(srs, evals, terms, log_blowup=1, shift=None, q=None, com=None):
    """Poly-IOP quotient Q = R(f(x), f(omega x)) / (X^n - 1) and [Q(tau)]_1.
    evals: (N, n, 8) device tensor of witness vectors on H; terms: list of
    (coefficient int < r, [factor indices]) with index a < N for f_a(x) and
    N <= a < 2N for f_(a-N)(omega x).  Returns (q (max(d - 1, 1) n, 8), com)."""
    torch = _torch()
    if (not isinstance(evals, torch.Tensor) or not evals.is_cuda or evals.dim() != 3 or evals.shape[2] != 8
            or evals.dtype != torch.int32 or not evals.is_contiguous()):
        raise TypeError("evals must be a contiguous int32 device tensor of shape (N, n, 8)")
    N, n = int(evals.shape[0]), int(evals.shape[1])
    L = n.bit_length() - 1
    if (1 << L) != n:
        raise ValueError("length must be a power of two")
    d = max((len(f) for _, f in terms), default=0)
    qlen = max(d - 1, 1) * n
    if q is None:
        q = torch.empty((qlen, 8), dtype=torch.int32, device=evals.device)
    elif q.shape[0] < qlen:
        raise ValueError("q needs %d rows" % qlen)
    if com is None:
        com = torch.empty((1, 16), dtype=torch.int32, device=evals.device)
    arr = _terms_array(terms)
    sp = None
    if shift is not None:
        sa, sp = _host_fr(shift)
    _check(lib.zk_quotient_polyiop(srs.handle, _ptr(evals), N, L, ctypes.cast(arr, ctypes.c_void_p), len(terms),
                                   int(log_blowup), sp, _ptr(q), _ptr(com), _stream(evals)))
    return q, com


def transcript_challenge(data, out=None):
    """Challenge (SHA-256(0||data) || SHA-256(1||data)) mod r of the bytes of
    the contiguous device tensor `data`.  Returns a (1, 8) device tensor."""
    torch = _torch()
    if not isinstance(data, torch.Tensor) or not data.is_cuda or not data.is_contiguous():
        raise TypeError("data must be a contiguous device tensor")
    if out is None:
        out = torch.empty((1, 8), dtype=torch.int32, device=data.device)
    nbytes = data.numel() * data.element_size()
    _check(lib.zk_transcript_challenge(_ptr(data) if nbytes else None, nbytes, _ptr(out), _stream(data)))
    return out


def acc_fold(gamma, C, C2, E, E2, Ej=None, v=None, v2=None, e=None, e2=None, ej=None):
    """One accumulation step: returns (C_out, E_out, v_out, e_out) for
    acc = (C, E, v, e) weighted by gamma and acc' = (C2, E2, v2, e2).
    C, C2: (k, 16); E, E2: (1, 16); Ej: (d - 1, 16) or None; v, v2: (len_v, 8)
    or None; e, e2: (len_e, 8) or None; ej: (d - 1, len_e, 8) or None;
    gamma: (1, 8) device Fr."""
    torch = _torch()
    gamma = _dev_words(gamma, 8, "gamma")
    C, C2 = _dev_words(C, 16, "C"), _dev_words(C2, 16, "C2")
    E, E2 = _dev_words(E, 16, "E"), _dev_words(E2, 16, "E2")
    k = C.shape[0]
    if C2.shape[0] != k:
        raise ValueError("C and C2 differ in length")
    d = 1 + (0 if Ej is None else int(Ej.shape[0]))
    ejp = None
    if Ej is not None and d > 1:
        Ej = _dev_words(Ej, 16, "Ej")
    dev = C.device
    C_out = torch.empty_like(C)
    E_out = torch.empty((1, 16), dtype=torch.int32, device=dev)
    len_v = 0 if v is None else int(v.shape[0])
    v_out = None
    if len_v:
        v, v2 = _dev_words(v, 8, "v"), _dev_words(v2, 8, "v2")
        v_out = torch.empty_like(v)
    len_e = 0 if e is None else int(e.shape[0])
    e_out = None
    if len_e:
        e, e2 = _dev_words(e, 8, "e"), _dev_words(e2, 8, "e2")
        e_out = torch.empty_like(e)
        if d > 1:
            if ej is None or tuple(ej.shape) != (d - 1, len_e, 8) or not ej.is_contiguous():
                raise ValueError("ej must be a contiguous (d - 1, len_e, 8) tensor")
            ejp = _ptr(ej)

    def p(t):
        return _ptr(t) if t is not None and t.numel() else None
    _check(lib.zk_acc_fold(k, p(C), p(C2), d, _ptr(E), _ptr(E2), p(Ej) if d > 1 else None, len_v, p(v), p(v2),
                           len_e, p(e), p(e2), ejp, _ptr(gamma), p(C_out), _ptr(E_out), p(v_out), p(e_out),
                           _stream(E)))
    return C_out, E_out, v_out, e_out


def srs_g2_setup(tau, n, device="cuda"):
    """[tau^i]_2 for i < n: (n, 32) device tensor (x0 x1 y0 y1 words)."""
    torch = _torch()
    out = torch.empty((int(n), 32), dtype=torch.int32, device=device)
    ta, tp = _host_fr(tau)
    _check(lib.zk_srs_g2_setup(tp, int(n), _ptr(out), _stream(out)))
    return out


class SRSG2:
    """A prepared G2 SRS (zk_srs_g2 handle) built from device points (n, 32)."""

    def __init__(self, points):
        points = _dev_words(points, 32, "points")
        h = ctypes.c_void_p()
        _check(lib.zk_srs_g2_create(_ptr(points), points.shape[0], ctypes.byref(h), _stream(points)))
        self.handle = h
        self.n = int(lib.zk_srs_g2_size(h))

    def close(self):
        if self.handle:
            _check(lib.zk_srs_g2_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def msm_g2_srs(srs, scalars, n=None, out=None):
    scalars = _dev_words(scalars, 8, "scalars")
    n = int(n if n is not None else scalars.shape[0])
    if n > scalars.shape[0]:
        raise ValueError("n exceeds the scalars")
    if out is None:
        out = _torch().empty((1, 32), dtype=_torch().int32, device=scalars.device)
    _check(lib.zk_msm_g2_srs(srs.handle, _ptr(scalars), n, _ptr(out), _stream(scalars)))
    return out


def fold(inst, gammas, out=None):
    """inst: (m, k, 16) device tensor; gammas: (m - 1, 8) device tensor."""
    torch = _torch()
    if inst.dim() != 3 or inst.shape[2] != 16 or inst.dtype != torch.int32 or not inst.is_contiguous():
        raise TypeError("inst must be a contiguous int32 tensor of shape (m, k, 16)")
    m, k = int(inst.shape[0]), int(inst.shape[1])
    if out is None:
        out = torch.empty((k, 16), dtype=torch.int32, device=inst.device)
    gp = ctypes.c_void_p(0)
    if m > 1:
        gammas = _dev_words(gammas, 8, "gammas")
        if gammas.shape[0] != m - 1:
            raise ValueError("need m - 1 challenges")
        gp = _ptr(gammas)
    _check(lib.zk_fold(_ptr(inst), gp, m, k, _ptr(out), _stream(inst)))
    return out


def msm_srs_workspace_bytes(srs, n):
    """Scratch bytes of one n-point commitment (host-only query)."""
    return int(lib.zk_msm_srs_workspace_bytes(srs.handle if srs is not None else None, int(n)))


def ntt_workspace_bytes(log_n):
    """Scratch bytes of one 2^log_n-point transform (host-only query)."""
    return int(lib.zk_ntt_workspace_bytes(int(log_n)))


def set_scratch_budget(nbytes):
    """Cap the library's scratch on the current device (0: no cap); a call
    whose scratch would exceed it raises ZkError with code ZK_EBUDGET."""
    _check(lib.zk_set_scratch_budget(int(nbytes)))


def scratch_held():
    """Scratch bytes the library holds on the current device (cache included)."""
    return int(lib.zk_scratch_held())


def release_cached_memory():
    """Free the library's cached scratch blocks on the current device."""
    _check(lib.zk_release_cached_memory())


# ---------------------------------------------------------------- observability

def calibrate_mad_rate(blocks=2048, iters=4096):
    """Sustained v_mad_u64_u32 products per second on the current device."""
    torch = _torch()
    rate = ctypes.c_double()
    _check(lib.zk_calibrate_mad_rate(int(blocks), int(iters), ctypes.byref(rate),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return rate.value


def profile_enable(on=True):
    _check(lib.zk_profile_enable(1 if on else 0))


def set_validate(on=True):
    """Check inputs (canonical Fr, on-curve G1) on the device before every call."""
    _check(lib.zk_set_validate(1 if on else 0))


def profile_only(region=None):
    """Record only regions called `region` (None: every region)."""
    _check(lib.zk_profile_only(region.encode() if region is not None else None))


def profile_read(region, reset=True):
    """(total milliseconds, number of regions) recorded for `region`."""
    ms = ctypes.c_double()
    cnt = ctypes.c_uint64()
    _check(lib.zk_profile_read(region.encode(), ctypes.byref(ms), ctypes.byref(cnt), 1 if reset else 0))
    return ms.value, cnt.value
