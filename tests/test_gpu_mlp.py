"""GPU tests of the warm-start MLP kernels (bf16 MFMA products, FP32 GELU,
MSE, Adam) against the float64 oracle with the same bfloat16 rounding
points, and of the learned warm start against plain VQE.

Tolerances: the oracle rounds the same operands to bfloat16 but accumulates
in float64 and evaluates GELU in float64; an FP32 accumulation can land a
value on the other side of a bfloat16 rounding boundary, which changes that
element by up to 2^-8 relative and propagates.  Outputs and gradients are
therefore compared at 1e-2 of their largest magnitude (a wrong fragment
layout or a missing term gives O(1) differences), losses at 1e-3 relative."""
import numpy as np
import pytest

from oracle import mlp as NN

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("widths,B", [([37, 256, 256, 360], 160), ([5, 7, 6, 4], 9),
                                      ([3, 33, 17], 1), ([16, 16], 16)])
def test_forward_matches_oracle(widths, B):
    from paper_2311_01242_amd.mlp import MLP
    rng = np.random.default_rng(len(widths) * 100 + B)
    p = _f32(NN.init_params(widths, 3) + rng.normal(0, 0.05, NN.n_params(widths)))
    x = _f32(rng.normal(size=(B, widths[0])))
    net = MLP(widths)
    net.set_params(p)
    assert np.array_equal(_f32(net.get_params()), p)
    y = net.forward(x).astype(np.float64)
    ref, _ = NN.forward(p, widths, x, rounding=True)
    assert np.abs(y - ref).max() <= 1e-2 * np.abs(ref).max()
    # and far from the unrounded network only by bfloat16-sized effects
    ref64, _ = NN.forward(p, widths, x, rounding=False)
    assert np.abs(y - ref64).max() <= 5e-2 * np.abs(ref64).max()


@pytest.mark.parametrize("widths,B", [([37, 256, 256, 360], 160), ([5, 7, 6, 4], 9)])
def test_loss_and_gradient_match_oracle(widths, B):
    from paper_2311_01242_amd.mlp import MLP
    rng = np.random.default_rng(7)
    p = _f32(NN.init_params(widths, 5))
    x = _f32(rng.normal(size=(B, widths[0])))
    y = _f32(rng.normal(0, 0.3, size=(B, widths[-1])))
    net = MLP(widths)
    net.set_params(p)
    loss, g = net.loss_grad(x, y)
    ref_loss, ref_g = NN.loss_and_grad(p, widths, x, y, rounding=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    for W_ref, W_got in zip(NN.unpack(ref_g, widths), NN.unpack(g.astype(np.float64), widths)):
        for a, b in zip(W_ref, W_got):
            assert np.abs(a - b).max() <= 1e-2 * max(np.abs(a).max(), 1e-30)


def test_adam_training_matches_oracle_and_decreases_loss():
    from paper_2311_01242_amd.mlp import MLP
    widths = [6, 32, 32, 5]
    rng = np.random.default_rng(11)
    p = _f32(NN.init_params(widths, 2))
    x = _f32(rng.normal(size=(40, 6)))
    y = _f32(np.tanh(x[:, :5] * 0.7) * 0.2)
    net = MLP(widths)
    net.set_params(p)
    lr = 1e-3
    trace = net.train(x, y, 3, lr=lr)
    # oracle: three Adam steps on the rounded network
    q, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    losses = []
    for t in range(1, 4):
        l, g = NN.loss_and_grad(q, widths, x, y, rounding=True)
        losses.append(l)
        q, m, v = NN.adam_step(q, g, m, v, t, lr=lr)
    assert np.allclose(trace, losses, rtol=1e-3, atol=0)
    d = np.abs(net.get_params().astype(np.float64) - q)
    # Adam normalises each gradient entry, so an entry whose gradient sits
    # near zero can move by up to lr * steps in either implementation
    assert d.max() <= 2.0 * 3 * lr
    assert np.median(d) <= 1e-2 * lr
    long = net.train(x, y, 1500, lr=lr)
    assert long[-1] < 0.05 * trace[0]


def test_rejects_bad_arguments():
    import paper_2311_01242_amd as vq
    from paper_2311_01242_amd.mlp import MLP
    net = MLP([4, 8, 2])
    with pytest.raises(vq.VQEError):
        net.forward(np.full((3, 4), np.nan))
    with pytest.raises(vq.VQEError):
        net.set_params(np.full(net.n_params, np.inf))
    with pytest.raises(vq.VQEError):
        net.train(np.zeros((3, 4)), np.zeros((3, 2)), 2, lr=-1.0)


def test_warm_start_beats_hf_start_on_a_small_scan():
    """8-qubit analogue of the learned warm start: 40 scan points of
    h, g = A + B e^-lam + C e^-2lam, 32 train / 8 held out.  The warm start
    must reach the plain-VQE energy (within 1 mHa) at every held-out point,
    and in fewer BFGS iterations on average (iterations to within 1 mHa of
    the lower of the two final energies; every run converged)."""
    from paper_2311_01242_amd import warmstart as W
    from vqe_inputs import warmstart_integrals
    n, ne = 8, 4
    fam = warmstart_integrals(n, 5)
    lams = np.linspace(0.7, 3.0, 40)
    A, scan = W.run_scan(fam, n, ne, lams)
    train, held = W.split(len(lams))
    net, norm, loss = W.train_warmstart(scan, train, steps=3000)
    assert loss[-1] < loss[0]
    rows = W.evaluate(scan, held, net, norm, A, n, ne, fam)
    s = W.summarize(rows)
    print(s)
    assert s["plain_converged"] == len(held) and s["warm_converged"] == len(held)
    assert s["warm_within_1mHa_of_plain"] == len(held)
    assert s["warm_iters_to_1mHa"]["missing"] == 0
    assert s["warm_iters_to_1mHa"]["mean"] < s["plain_iters_to_1mHa"]["mean"]
