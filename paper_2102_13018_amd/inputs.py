"""Seeded synthetic inputs for the star-forest workloads.

This module holds graph and data generators only: none of the SF
operations' arithmetic lives here.  Both the GPU path (tests, benchmark) and
the CPU oracle consume what it produces.  Every generator is driven by
``numpy.random.default_rng(seed)`` (PCG64) and is therefore reproducible.

A star forest is returned as a :class:`Graph`: ``nroots``; ``iroot[i]``, the
root of leaf i; ``ilocal`` (``None`` when the leaf space is contiguous, as in
the paper's PetscSFSetGraph with local = NULL, Section 3.1); ``ranks[i]``, the
segment label of leaf i (the would-be neighbour that owns the leaf's root);
and ``leafspace``, the number of slots of the leaf buffer.

Workloads (stand-ins for the paper's uses of PetscSF):
  * :func:`fig2`            -- the three-rank example of Fig. 2, flattened;
  * :func:`single_sf`       -- one SF, uniform roots, permuted leaf slots;
  * :func:`halo3d`          -- periodic ghost layer of an n^3 box (Section 5.2
                               multi-strided patterns, 27-point stencil);
  * :func:`spmv_ghost`      -- Zipf root in-degree, 64 neighbour segments
                               (SpMV ghost SF of Section 4.1);
  * :func:`batch_mix`       -- many small uneven SFs (Section 5.4 launch
                               costs);
  * :func:`knn_graph`       -- k-nearest-neighbour mesh graph (DMPlex-style
                               ghost exchange and assembly, Section 4.2);
  * :func:`split_matrix`    -- one rank's diagonal / off-diagonal CSR blocks
                               and ghost SF of a row-distributed sparse
                               matrix (SpMV, Section 4.1).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

PAIR = np.dtype([("v", "<f8"), ("i", "<i4"), ("pad", "<i4")])


@dataclass
class Graph:
    nroots: int
    iroot: np.ndarray                  # int64 [nleaves]
    ilocal: Optional[np.ndarray]       # int64 [nleaves] or None
    ranks: np.ndarray                  # int64 [nleaves], segment label per leaf
    leafspace: int
    meta: dict = field(default_factory=dict)

    @property
    def nleaves(self):
        return int(self.iroot.size)


# ------------------------------------------------------------------ Fig. 2
def fig2():
    """Fig. 2 of the paper flattened onto one device.

    Roots: rank 0 -> 0..2, rank 1 -> 3..6, rank 2 -> 7..8 (nroots = 9).
    Leaf slots: rank 0 -> 0..3, rank 1 -> 4..7, rank 2 -> 8..10; slot 6 is
    rank 1's isolated leaf (a hole).  The remote (rank, offset) pairs of the
    figure become global root indices; the leaf's own rank is the segment.
    """
    root_base = {0: 0, 1: 3, 2: 7}
    leaf_base = {0: 0, 1: 4, 2: 8}
    # (leaf rank, local leaf index, root rank, root offset) as printed in Fig. 2
    edges = [(0, 0, 1, 2), (0, 1, 1, 0), (0, 2, 1, 0), (0, 3, 0, 2),
             (1, 0, 2, 0), (1, 1, 0, 0), (1, 3, 2, 1),
             (2, 0, 0, 0), (2, 1, 1, 0), (2, 2, 1, 3)]
    ilocal = np.array([leaf_base[lr] + li for lr, li, _, _ in edges], dtype=np.int64)
    iroot = np.array([root_base[rr] + ro for _, _, rr, ro in edges], dtype=np.int64)
    ranks = np.array([lr for lr, _, _, _ in edges], dtype=np.int64)
    return Graph(9, iroot, ilocal, ranks, 11, {"name": "fig2"})


# ------------------------------------------------------ single uniform SF
def single_sf(seed=1, nroots=4096, nleaves=16384, leafspace=20000):
    """One SF: roots uniform in [0, nroots); leaf slots a random subset
    (in random order) of [0, leafspace)."""
    rng = np.random.default_rng(seed)
    iroot = rng.integers(0, nroots, size=nleaves, dtype=np.int64)
    ilocal = rng.permutation(leafspace)[:nleaves].astype(np.int64)
    ranks = np.zeros(nleaves, dtype=np.int64)
    return Graph(nroots, iroot, ilocal, ranks, leafspace,
                 {"name": f"single_sf(nroots={nroots},nleaves={nleaves},leafspace={leafspace})",
                  "seed": seed})


# ------------------------------------------------------------- 3-D halo
HALO_DIRS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
             if (dz, dy, dx) != (0, 0, 0)]


def halo3d(n=256):
    """Periodic ghost layer (width 1) of an owned n^3 box, 27-point stencil.

    Roots are the owned points, index x + n*y + n*n*z.  Leaves are the ghost
    points, grouped into 26 segments (one per neighbour direction, in
    lexicographic (dz, dy, dx) order), each packed x-fastest into one
    contiguous leaf buffer.  A ghost at (x, y, z) with coordinates in
    [-1, n] maps to the owned point (x mod n, y mod n, z mod n), i.e. the
    opposite face of the periodic box.
    """
    iroot, ranks = [], []
    for s, (dz, dy, dx) in enumerate(HALO_DIRS):
        def rng1(d):
            return np.array([-1]) if d < 0 else (np.array([n]) if d > 0 else np.arange(n))
        zs, ys, xs = rng1(dz), rng1(dy), rng1(dx)
        z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")  # x fastest in C order
        r = (x % n) + n * (y % n) + n * n * (z % n)
        iroot.append(r.ravel().astype(np.int64))
        ranks.append(np.full(r.size, s, dtype=np.int64))
    iroot = np.concatenate(iroot)
    ranks = np.concatenate(ranks)
    return Graph(n ** 3, iroot, None, ranks, iroot.size, {"name": f"halo3d(n={n})", "n": n})


# ---------------------------------------------------------- SpMV ghost SF
def _segment_sizes(rng, total, nseg, spread=1000.0):
    """nseg log-uniform weights exp(U(0, ln spread)) scaled to sum exactly to
    total by largest remainder, each at least 1."""
    w = np.exp(rng.uniform(0.0, np.log(spread), size=nseg))
    q = w / w.sum() * (total - nseg)
    base = np.floor(q).astype(np.int64)
    rem = (total - nseg) - base.sum()
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return base + 1


def spmv_ghost(seed=3, nroots=2_000_000, nleaves=16_000_000, zipf_s=1.1, nseg=64):
    """Unstructured SpMV-ghost SF.

    Root popularity is Zipf: the root of popularity rank k (1-based) is drawn
    with probability proportional to k^-s; ranks map to root ids through a
    seeded permutation.  Each leaf draws its root independently.  Leaves are
    contiguous (ilocal = None) and split into ``nseg`` contiguous neighbour
    segments of log-uniform size.
    """
    rng = np.random.default_rng(seed)
    p = np.arange(1, nroots + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(nleaves)
    rank = np.searchsorted(cdf, u, side="right")
    np.minimum(rank, nroots - 1, out=rank)
    perm = rng.permutation(nroots)
    iroot = perm[rank].astype(np.int64)
    sizes = _segment_sizes(rng, nleaves, min(nseg, nleaves)) if nleaves else np.zeros(0, np.int64)
    ranks = np.repeat(np.arange(sizes.size, dtype=np.int64), sizes)
    return Graph(nroots, iroot, None, ranks, nleaves,
                 {"name": f"spmv_ghost(nroots={nroots},nleaves={nleaves},zipf={zipf_s})",
                  "seed": seed})


# --------------------------------------------------------------- batches
def batch_mix(seed=4, count=64, lmin=1e3, lmax=1e6):
    """``count`` independent SFs of uneven size, unit and operation.

    nleaves ~ floor(exp(U(ln lmin, ln lmax))), nroots = floor(nleaves /
    U{1..8}) (at least 1), roots uniform, ilocal = None, block size U{1..8},
    dtype U{float64, float32, int32}, op U{bcast-replace, reduce-sum}.
    """
    rng = np.random.default_rng(seed)
    items = []
    dtypes = [np.float64, np.float32, np.int32]
    for k in range(count):
        nl = int(np.floor(np.exp(rng.uniform(np.log(lmin), np.log(lmax)))))
        nl = max(nl, 1)
        nr = max(1, nl // int(rng.integers(1, 9)))
        iroot = rng.integers(0, nr, size=nl, dtype=np.int64)
        bs = int(rng.integers(1, 9))
        dt = np.dtype(dtypes[int(rng.integers(0, 3))])
        kind = "bcast" if int(rng.integers(0, 2)) == 0 else "reduce"
        g = Graph(nr, iroot, None, np.zeros(nl, np.int64), nl, {"name": f"batch[{k}]"})
        items.append({"graph": g, "bs": bs, "dtype": dt, "kind": kind,
                      "op": "replace" if kind == "bcast" else "sum",
                      "seed": int(rng.integers(0, 2 ** 31))})
    return items


# ----------------------------------------------------------- k-NN graph
def knn_graph(seed=5, npoints=1_000_000, k=8):
    """k-nearest-neighbour graph of points uniform in the unit cube.

    Leaf k*i + j is connected to root = the j-th nearest neighbour of point i
    (self excluded, ties by index as returned by the KD-tree).  ilocal = None.
    """
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((npoints, 3))
    tree = cKDTree(pts)
    _, nb = tree.query(pts, k=k + 1, workers=-1)
    if not np.array_equal(nb[:, 0], np.arange(npoints)):
        raise RuntimeError("coincident points: nearest neighbour is not the point itself")
    nb = nb[:, 1:]
    iroot = nb.reshape(-1).astype(np.int64)
    ranks = np.zeros(iroot.size, np.int64)
    return Graph(npoints, iroot, None, ranks, iroot.size,
                 {"name": f"knn(npoints={npoints},k={k})", "seed": seed})


# --------------------------------------------------------------- data
def split_matrix(seed=7, n=1_000_000, nnz_a=15, m=250_000, nnz_b=4):
    """One rank's share of a row-distributed sparse matrix (Section 4.1,
    Fig. 3's kind): the diagonal block A (n x n CSR: the diagonal plus
    nnz_a - 1 random columns per row), the off-diagonal block B (n x m CSR
    over the ghost vector lvec, nnz_b random columns per row, reduced local
    column indices), values N(0,1), and the ghost SF: lvec entry j is a leaf
    of root iroot[j], m distinct roots of the n (the owners' local indices of
    the ghost columns; on one device every root is local).  A stand-in for
    the SuiteSparse matrices the paper times, which are not used.
    Returns a dict with n, m, A = (rowptr, colidx, values), B, iroot."""
    rng = np.random.default_rng(seed)

    def csr(nrows, ncols, per_row, diag):
        cols = rng.integers(0, ncols, (nrows, per_row), dtype=np.int64)
        if diag:
            cols[:, 0] = np.arange(nrows)
        cols.sort(axis=1)
        rowptr = np.arange(nrows + 1, dtype=np.int64) * per_row
        vals = rng.standard_normal(nrows * per_row)
        return rowptr, cols.reshape(-1).astype(np.int32), vals

    A = csr(n, n, nnz_a, True)
    B = csr(n, m, nnz_b, False)
    iroot = np.sort(rng.choice(n, m, replace=False)).astype(np.int64)
    rng.shuffle(iroot)
    return {"n": n, "m": m, "A": A, "B": B, "iroot": iroot,
            "meta": {"name": f"split_matrix(n={n}, nnz_a={nnz_a}, m={m}, nnz_b={nnz_b})", "seed": seed}}


def normal(rng, shape, dtype=np.float64):
    return rng.standard_normal(shape).astype(dtype)


def unit_data(rng, n, bs, dtype, kind="normal"):
    """Data for n units of bs elements: N(0,1) for floats, U[-1000,1000) for
    int32 (``kind='small'``), full-range for ``kind='full'``."""
    shape = (n,) if bs == 1 else (n, bs)
    dtype = np.dtype(dtype)
    if dtype.kind == "f":
        return rng.standard_normal(shape).astype(dtype)
    info = np.iinfo(dtype)
    if kind == "full":
        return rng.integers(info.min, info.max, size=shape, dtype=dtype, endpoint=True)
    if kind == "u100":
        return rng.integers(0, 100, size=shape, dtype=dtype)
    return rng.integers(-1000, 1000, size=shape, dtype=dtype)


def bf16_bits(rng, n, bs=1, scale=1.0):
    """bfloat16 data as 16-bit patterns (np.uint16): N(0, scale^2) binary32
    values with the low 16 bits cleared, so every value is a bfloat16."""
    shape = (n,) if bs == 1 else (n, bs)
    x = (rng.standard_normal(shape) * scale).astype(np.float32)
    return (x.view(np.uint32) >> 16).astype(np.uint16)


def maxloc_leaves(rng, nleaves, ties=False):
    """MAXLOC leaf units: v ~ N(0,1) (quantised to 1/4 when ``ties``), i = leaf index."""
    a = np.zeros(nleaves, dtype=PAIR)
    v = rng.standard_normal(nleaves)
    if ties:
        v = np.round(v * 4.0) / 4.0
    a["v"] = v
    a["i"] = np.arange(nleaves, dtype=np.int32)
    return a


def maxloc_roots(rng, nroots, ties=False):
    """MAXLOC root units: v ~ N(0,1) (quantised when ``ties``), i = -1."""
    a = np.zeros(nroots, dtype=PAIR)
    v = rng.standard_normal(nroots)
    if ties:
        v = np.round(v * 4.0) / 4.0
    a["v"] = v
    a["i"] = -1
    return a
