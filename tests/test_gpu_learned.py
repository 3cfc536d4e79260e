"""GPU parity of the parameter chooser's kernels: features and the network.

The paper has no learned component (parity unpinned by the paper); the bars
come from the arithmetic: fp64 row statistics agree to 1e-6 relative after the
cast to fp32; the fp32 Arnoldi features agree to 2e-3 absolute (they are
log10 values and normalised Ritz-value ratios of an fp32 process); the fp32
network agrees with the fp64 oracle to 1e-5 relative in the output and 1e-4
relative in the gradient (5443 parameters, sums over at most 64 samples).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import features as F
from oracle import mlp as OM
from paper_2109_01232_amd import binding as B
from paper_2109_01232_amd import problems as P

from gpu_common import dev_tensor, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.lib()


@pytest.mark.parametrize("case", ["conv64", "aniso3d", "varcoef27", "chooser", "cyclic"])
def test_features_match_oracle(case):
    if case == "conv64":
        s = P.parity_system()
        A, b = s.A, s.b
    elif case == "aniso3d":
        A = P.conv_diff(3, 15, 10.0, (1, 1, 1), (1, 1, 1e-2))
        b = A.scipy() @ np.random.default_rng(0).uniform(-1, 1, A.n)
    elif case == "varcoef27":
        A = P.varcoef27(12, 2)
        b = A.scipy() @ np.random.default_rng(1).uniform(-1, 1, A.n)
    elif case == "chooser":
        sysm = P.chooser_system(5, n_max=3e4)
        A, b = sysm.A, sysm.b
    else:
        # seven known eigenvalues, exact fp32 Arnoldi ending in an exact breakdown
        from test_oracle_features import cyclic_system

        A, _, b = cyclic_system()
    say("features", case)
    M = B.Matrix.from_csr(A)
    got = B.gmresir_features(M, dev_tensor(b))
    ref = F.features(A, b)
    assert np.allclose(got[:10], ref[:10], rtol=1e-6, atol=1e-6), (got[:10], ref[:10])
    assert np.allclose(got[10:], ref[10:], atol=2e-3), (got[10:], ref[10:])


def _net_inputs(seed, batch):
    rng = np.random.default_rng(seed)
    p = OM.init_params(seed) + rng.normal(0, 0.05, OM.NPARAM)
    X = rng.standard_normal((batch, 16)) * 3.0 + 1.0
    T = rng.standard_normal((batch, 3))
    shift = rng.standard_normal(16)
    scale = rng.uniform(0.2, 1.5, 16)
    return p, X, T, shift, scale


@pytest.mark.parametrize("batch", [1, 7, 64, 333])
def test_mlp_forward(batch):
    p, X, T, shift, scale = _net_inputs(batch, batch)
    say("mlp forward", batch)
    f32 = lambda a: dev_tensor(np.asarray(a, dtype=np.float32))
    Y = torch.empty((batch, 3), dtype=torch.float32, device="cuda")
    B.gmresir_mlp_forward(f32(p), f32(shift), f32(scale), f32(X), Y)
    torch.cuda.synchronize()
    ref = OM.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
                     shift.astype(np.float32), scale.astype(np.float32))
    assert rel(Y.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("batch", [1, 33, 200])
def test_mlp_gradient(batch):
    p, X, T, shift, scale = _net_inputs(100 + batch, batch)
    say("mlp grad", batch)
    f32 = lambda a: dev_tensor(np.asarray(a, dtype=np.float32))
    g = torch.empty(OM.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    B.gmresir_mlp_loss_grad(f32(p), f32(shift), f32(scale), f32(X), f32(T), g, loss)
    torch.cuda.synchronize()
    c = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    lref, gref = OM.loss_and_grad(c(p), c(X), c(T), c(shift), c(scale))
    assert abs(loss.item() - lref) <= 1e-5 * lref
    assert rel(g.cpu().numpy(), gref) <= 1e-4
    assert np.allclose(g.cpu().numpy(), gref, rtol=1e-3, atol=1e-6 * np.abs(gref).max())


def test_mlp_adam_step_and_training():
    p, X, T, shift, scale = _net_inputs(7, 128)
    T = np.tanh(X[:, :3] * 0.3)
    f32 = lambda a: dev_tensor(np.asarray(a, dtype=np.float32))
    P_ = f32(p)
    m = torch.zeros(OM.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    Xd, Td, sh, sc = f32(X), f32(T), f32(shift), f32(scale)
    say("adam step 1")
    B.gmresir_mlp_train_step(P_, m, v, sh, sc, Xd, Td, 1e-3, 1, loss)
    torch.cuda.synchronize()
    c = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    l0, g = OM.loss_and_grad(c(p), c(X), c(T), c(shift), c(scale))
    p1, m1, v1 = OM.adam_step(c(p), g, np.zeros(OM.NPARAM), np.zeros(OM.NPARAM), 1, 1e-3)
    assert abs(loss.item() - l0) <= 1e-5 * l0
    assert rel(m.cpu().numpy(), m1) <= 1e-4
    assert rel(v.cpu().numpy(), v1) <= 2e-4
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.allclose(P_.cpu().numpy()[big], p1[big], atol=2e-6)
    say("adam training 300 steps")
    for step in range(2, 302):
        B.gmresir_mlp_train_step(P_, m, v, sh, sc, Xd, Td, 1e-2, step, loss)
    torch.cuda.synchronize()
    assert loss.item() < 0.1 * l0
