"""GPU tests of the differentiable gather/scatter: SFBcast forward with
SFReduce(SUM) backward and the reverse, checked against the oracle's adjoint
(bit-exact on the deterministic path) and against FP64 central finite
differences of a 3-layer checkpointed chain on a k-NN graph."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2102_13018_amd import autograd as A
from paper_2102_13018_amd import inputs
from paper_2102_13018_amd import sf as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def knn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = inputs.knn_graph(seed=5, npoints=10000, k=8)
    sf = S.StarForest(g.nroots, g.iroot, None, None).setup(reduce_mode="deterministic")
    return g, A.DiffSF(sf, g.nleaves)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_backward_matches_oracle_adjoint(knn, dtype):
    g, dsf = knn
    rng = np.random.default_rng(1)
    npd = np.float32 if dtype == torch.float32 else np.float64
    h = torch.from_numpy(rng.standard_normal((g.nroots, 16)).astype(npd)).cuda().requires_grad_(True)
    gleaf = rng.standard_normal((g.nleaves, 16)).astype(npd)
    leaf = A.sf_bcast(dsf, h)
    leaf.backward(torch.from_numpy(gleaf).cuda())
    want = oracle.reduce(g.nroots, g.iroot, None, gleaf, np.zeros((g.nroots, 16), npd), "sum")
    assert h.grad.cpu().numpy().tobytes() == want.tobytes()
    # the reverse pair: d leaf of Reduce SUM is Bcast of the upstream gradient
    m = torch.from_numpy(rng.standard_normal((g.nleaves, 16)).astype(npd)).cuda().requires_grad_(True)
    r0 = torch.zeros((g.nroots, 16), dtype=dtype, device="cuda", requires_grad=True)
    gout = rng.standard_normal((g.nroots, 16)).astype(npd)
    out = A.sf_reduce_sum(dsf, m, r0)
    out.backward(torch.from_numpy(gout).cuda())
    want = oracle.bcast(g.nroots, g.iroot, None, gout, np.zeros((g.nleaves, 16), npd))
    assert m.grad.cpu().numpy().tobytes() == want.tobytes()
    assert r0.grad.cpu().numpy().tobytes() == gout.tobytes()


def test_forward_matches_oracle(knn):
    g, dsf = knn
    rng = np.random.default_rng(2)
    h = rng.standard_normal((g.nroots, 16)).astype(np.float32)
    a = (rng.standard_normal(g.nleaves) / np.sqrt(8)).astype(np.float32)
    got = A.layer(dsf, torch.from_numpy(h).cuda(), torch.from_numpy(a).cuda()).cpu().numpy()
    e = oracle.bcast(g.nroots, g.iroot, None, h, np.zeros((g.nleaves, 16), np.float32))
    z = oracle.reduce(g.nroots, g.iroot, None, e * a[:, None], np.zeros((g.nroots, 16), np.float32))
    assert np.array_equal(got, np.tanh(z)) or np.allclose(got, np.tanh(z), rtol=0, atol=2e-7)
    # the SF part is exact: compare pre-activations through atanh-free route
    zz = A.sf_reduce_sum(dsf, A.sf_bcast(dsf, torch.from_numpy(h).cuda()) * torch.from_numpy(a).cuda()[:, None],
                         torch.zeros((g.nroots, 16), device="cuda")).cpu().numpy()
    assert zz.tobytes() == z.tobytes()


def test_chain_gradient_vs_finite_differences(knn):
    """FP64 central differences, eps = 1e-6, along 32 random directions and
    200 random coordinates: |fd - an| <= 1e-6 + 1e-5 |an|."""
    g, dsf = knn
    rng = np.random.default_rng(3)
    h0 = torch.from_numpy(rng.standard_normal((g.nroots, 16))).cuda()
    a = [torch.from_numpy(rng.standard_normal(g.nleaves) / np.sqrt(8)).cuda() for _ in range(3)]
    G = torch.from_numpy(rng.standard_normal((g.nroots, 16))).cuda()
    h = h0.clone().requires_grad_(True)
    loss = A.chain_loss(dsf, h, a, G, checkpoint=True)
    loss.backward()
    grad = h.grad.clone()

    def f(x):
        with torch.no_grad():
            return float(A.chain_loss(dsf, x, a, G, checkpoint=False))

    eps = 1e-6
    for _ in range(32):
        v = torch.from_numpy(rng.standard_normal((g.nroots, 16))).cuda()
        v /= v.norm()
        fd = (f(h0 + eps * v) - f(h0 - eps * v)) / (2 * eps)
        an = float((grad * v).sum())
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (fd, an)
    flat = grad.reshape(-1)
    for idx in rng.choice(flat.numel(), 200, replace=False):
        e = torch.zeros_like(h0).reshape(-1)
        e[idx] = 1.0
        e = e.reshape(h0.shape)
        fd = (f(h0 + eps * e) - f(h0 - eps * e)) / (2 * eps)
        an = float(flat[idx])
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (idx, fd, an)


def test_checkpointed_equals_plain(knn):
    g, dsf = knn
    rng = np.random.default_rng(4)
    h0 = torch.from_numpy(rng.standard_normal((g.nroots, 16)).astype(np.float32)).cuda()
    a = [torch.from_numpy((rng.standard_normal(g.nleaves) / np.sqrt(8)).astype(np.float32)).cuda() for _ in range(3)]
    G = torch.from_numpy(rng.standard_normal((g.nroots, 16)).astype(np.float32)).cuda()
    grads = []
    for ck in (True, False):
        h = h0.clone().requires_grad_(True)
        A.chain_loss(dsf, h, a, G, checkpoint=ck).backward()
        grads.append(h.grad.cpu().numpy())
    assert grads[0].tobytes() == grads[1].tobytes()     # deterministic path: identical bits
