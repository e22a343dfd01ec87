"""Shared helpers of the GPU parity tests: device copies of NumPy units
(including MAXLOC pairs, carried as raw bytes), the tolerance of the atomic
FP sum, and the validity check of atomic FetchAndOp chains."""
import numpy as np
import torch

from paper_2102_13018_amd import sf as S

PAIR = np.dtype([("v", "<f8"), ("i", "<i4"), ("pad", "<i4")])
BF16 = np.dtype([("bf16", "<u2")])     # bfloat16 patterns (the oracle's carrier dtype)


def sfdtype(a):
    a = np.asarray(a)
    if a.dtype == PAIR:
        return S.SF_F64_I32
    if a.dtype == BF16:
        return S.SF_BF16
    return {np.dtype(np.float64): S.SF_F64, np.dtype(np.float32): S.SF_F32,
            np.dtype(np.int32): S.SF_I32, np.dtype(np.int64): S.SF_I64,
            np.dtype(np.float16): S.SF_F16}[a.dtype]


def unit(a):
    a = np.asarray(a)
    bs = 1 if a.ndim == 1 else int(np.prod(a.shape[1:]))
    return S.SfUnit(sfdtype(a), bs)


def dev(a, offset_bytes=0):
    """Device copy of a NumPy array (raw bytes).  With offset_bytes the data
    start that many bytes into the allocation (to test alignment paths)."""
    a = np.ascontiguousarray(a)
    raw = a.view(np.uint8).reshape(-1)
    t = torch.empty(raw.size + offset_bytes + 16, dtype=torch.uint8, device="cuda")
    view = t[offset_bytes:offset_bytes + raw.size]
    view.copy_(torch.from_numpy(raw.copy()))
    return view


def host(t, like):
    """NumPy copy of a device byte buffer shaped like ``like``."""
    raw = t.cpu().numpy()
    like = np.asarray(like)
    return raw.view(like.dtype).reshape(like.shape).copy()


def same_bits(a, b):
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    if a.dtype == PAIR:
        return np.array_equal(a["v"].view(np.uint64), b["v"].view(np.uint64)) and np.array_equal(a["i"], b["i"])
    return a.shape == b.shape and a.tobytes() == b.tobytes()


def first_diff(a, b):
    """Up to ten positions where a and b differ bitwise, with both values."""
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    if a.dtype == PAIR:
        bad = np.nonzero((a["v"].view(np.uint64) != b["v"].view(np.uint64)) | (a["i"] != b["i"]))[0]
    else:
        bad = np.nonzero(a.view(f"u{a.itemsize}") != b.view(f"u{b.itemsize}"))[0]
    return bad[:10], a[bad[:10]], b[bad[:10]]


def atomic_sum_tolerance(got, want, root0, leaf_units, iroot, rtol):
    """|got - oracle| <= rtol * (|root0| + sum |x_i|) per root and element."""
    scale = np.abs(np.asarray(root0, dtype=np.float64)).copy()
    np.add.at(scale, iroot, np.abs(np.asarray(leaf_units, dtype=np.float64)))
    err = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(want, dtype=np.float64))
    return bool(np.all(err <= rtol * scale)), float((err / np.maximum(scale, 1e-300)).max())


def check_fetch_chain(iroot, slots, root0, leaf, fetched, root_final):
    """Validity of an atomic FetchAndOp SUM with non-negative integer leaves:
    the final root is root0 + sum of its leaves, and the leaves of every
    root, sorted by (fetched, value), form the chain f0 = root0,
    f[k+1] = f[k] + v[k], final = f[last] + v[last]."""
    iroot = np.asarray(iroot)
    v = np.asarray(leaf)[slots].astype(np.int64)
    f = np.asarray(fetched)[slots].astype(np.int64)
    r0 = np.asarray(root0).astype(np.int64)
    want = r0.copy()
    np.add.at(want, iroot, v)
    assert np.array_equal(np.asarray(root_final).astype(np.int64), want), "final roots"
    order = np.lexsort((v, f, iroot))
    ri, fi, vi = iroot[order], f[order], v[order]
    first = np.ones(ri.size, bool)
    first[1:] = ri[1:] != ri[:-1]
    assert np.array_equal(fi[first], r0[ri[first]]), "chain start"
    nxt = ~first[1:]
    assert np.array_equal(fi[1:][nxt], (fi[:-1] + vi[:-1])[nxt]), "chain links"
    last = np.ones(ri.size, bool)
    last[:-1] = ri[:-1] != ri[1:]
    assert np.array_equal(fi[last] + vi[last], want[ri[last]]), "chain end"


def check_fetch_chain_fp(iroot, slots, root0, leaf, fetched, root_final, rtol):
    """Validity of an atomic floating-point FetchAndOp SUM with leaves bounded
    away from 0 (so that rounding cannot reorder a root's fetched values):
    per root, sorted by fetched value, f0 = root0, f[k+1] = f[k] + v[k] and
    final = f[last] + v[last], each within rtol * (|root0| + sum |v|) of that
    root (the atomic-sum tolerance)."""
    iroot = np.asarray(iroot)
    v = np.asarray(leaf, dtype=np.float64)[slots]
    f = np.asarray(fetched, dtype=np.float64)[slots]
    r0 = np.asarray(root0, dtype=np.float64)
    rf = np.asarray(root_final, dtype=np.float64)
    scale = np.abs(r0).copy()
    np.add.at(scale, iroot, np.abs(v))
    order = np.lexsort((f, iroot))
    ri, fi, vi = iroot[order], f[order], v[order]
    tol = rtol * scale[ri]
    first = np.ones(ri.size, bool)
    first[1:] = ri[1:] != ri[:-1]
    assert np.all(np.abs(fi[first] - r0[ri[first]]) <= tol[first]), "chain start"
    nxt = ~first[1:]
    assert np.all(np.abs(fi[1:][nxt] - (fi[:-1] + vi[:-1])[nxt]) <= tol[1:][nxt]), "chain links"
    last = np.ones(ri.size, bool)
    last[:-1] = ri[:-1] != ri[1:]
    assert np.all(np.abs(fi[last] + vi[last] - rf[ri[last]]) <= tol[last]), "chain end"
