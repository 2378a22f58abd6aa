"""Differentiation form: the softmax-gated ensemble head (bias b over the vocabulary, gate theta over
{LLM, n-gram orders 1..4}).  The hand-written backward kernel behind a torch.autograd.Function is
checked against central finite differences (h = 1e-4, FP64) and the oracle's closed-form
gradient, to a norm-wise relative error of 1e-4; the ensemble pipeline matches the oracle and
round-trips."""
import numpy as np
import pytest

import synth
from oracle import pipeline as op
from oracle.head import EnsembleGate, softmax
from tests.nc_util import gpu_available, kl_bits, make_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not gpu_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(seed, rows=6, v=3000, nexp=5):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(rows, v)) * 0.7
    b = rng.normal(size=v) * 0.1
    theta = rng.normal(size=nexp) * 0.5
    P = np.stack([[softmax(rng.normal(size=v) * 2.0) for _ in range(nexp - 1)] for _ in range(rows)])
    t = rng.integers(0, v, size=rows)
    return z, b, theta, P, t


def _oracle_grads(z, b, theta, P, t):
    gth = np.zeros_like(theta)
    gb = np.zeros_like(b)
    loss = 0.0
    for r in range(z.shape[0]):
        q0 = softmax(np.log(softmax(z[r])) + b)
        g1, g2 = EnsembleGate.grads(theta, q0, list(P[r]), int(t[r]))
        gth += g1
        gb += g2
        loss += EnsembleGate.loss(theta, b, z[r], list(P[r]), int(t[r]))
    return loss, gb, gth


@pytest.mark.parametrize("seed", [0, 1])
def test_autograd_backward_matches_oracle_and_finite_differences(dev, seed):
    from paper_2602_19626_amd.ensemble import ensemble_loss
    z, b, theta, P, t = _case(seed)
    tz = torch.tensor(z, dtype=torch.float32, device=dev)
    tb = torch.tensor(b, dtype=torch.float32, device=dev, requires_grad=True)
    tth = torch.tensor(theta, dtype=torch.float32, device=dev, requires_grad=True)
    tP = torch.tensor(P, dtype=torch.float32, device=dev).contiguous()
    tt = torch.tensor(t, dtype=torch.int32, device=dev)
    loss = ensemble_loss(tz, tb, tth, tP, tt)
    loss.sum().backward()
    gb = tb.grad.double().cpu().numpy()
    gth = tth.grad.double().cpu().numpy()
    # closed-form oracle gradient on the float32-rounded inputs
    z32, b32, th32, P32 = (np.float64(np.float32(x)) for x in (z, b, theta, P))
    ref_loss, ref_gb, ref_gth = _oracle_grads(z32, b32, th32, P32, t)
    assert abs(float(loss.detach().sum()) - ref_loss) / abs(ref_loss) < 1e-5
    assert np.linalg.norm(gb - ref_gb) / np.linalg.norm(ref_gb) < 1e-4
    assert np.linalg.norm(gth - ref_gth) / np.linalg.norm(ref_gth) < 1e-4
    # central finite differences of the FP64 oracle loss (h = 1e-4)
    h = 1e-4
    fd_th = np.array([(_oracle_grads(z32, b32, th32 + h * e, P32, t)[0]
                       - _oracle_grads(z32, b32, th32 - h * e, P32, t)[0]) / (2 * h)
                      for e in np.eye(len(theta))])
    assert np.linalg.norm(gth - fd_th) / np.linalg.norm(fd_th) < 1e-4
    idx = np.unique(np.concatenate([t, np.arange(0, z.shape[1], 97)]))
    fd_b = []
    for i in idx:
        e = np.zeros_like(b32)
        e[i] = h
        fd_b.append((_oracle_grads(z32, b32 + e, th32, P32, t)[0]
                     - _oracle_grads(z32, b32 - e, th32, P32, t)[0]) / (2 * h))
    fd_b = np.array(fd_b)
    assert np.linalg.norm(gb[idx] - fd_b) / np.linalg.norm(fd_b) < 1e-4


def test_sgd_step_in_place(dev):
    from paper_2602_19626_amd.ensemble import ensemble_sgd_step
    z, b, theta, P, t = _case(5)
    tz = torch.tensor(z, dtype=torch.float32, device=dev)
    tb = torch.tensor(b, dtype=torch.float32, device=dev)
    tth = torch.tensor(theta, dtype=torch.float32, device=dev)
    tP = torch.tensor(P, dtype=torch.float32, device=dev).contiguous()
    tt = torch.tensor(t, dtype=torch.int32, device=dev)
    ensemble_sgd_step(tz, tb, tth, tP, tt, lr=1e-3)
    z32, b32, th32, P32 = (np.float64(np.float32(x)) for x in (z, b, theta, P))
    _, gb, gth = _oracle_grads(z32, b32, th32, P32, t)
    assert np.max(np.abs(tb.double().cpu().numpy() - (b32 - 1e-3 * gb))) < 1e-6
    assert np.max(np.abs(tth.double().cpu().numpy() - (th32 - 1e-3 * gth))) < 1e-6


def test_ensemble_pipeline_matches_oracle_and_roundtrips(dev):
    import dataclasses
    wl = dataclasses.replace(synth.WORKLOADS["tiny"], ensemble=True, skip="none", ngram_order=4)
    toks = synth.workload_streams(wl, max_len=800)[0]
    ctx, w = make_context(wl, max_streams=1)
    pos = [0, 1, 50, 200, 450, 799]
    orc = op.encode(op.Settings.from_workload(wl), wl.shape, w, toks, record=pos, block=1,
                    quantize=False)
    ctx.reset(1, len(toks) + 1)
    for i in pos:
        p, pr = ctx.probs_for_context(0, toks[:i], probe=True)
        assert pr["mode"] == op.MODE_ENSEMBLE
        assert kl_bits(orc.records[i]["p"], p) < 1e-6, i
    data, bits = ctx.encode_stream([toks])
    assert np.array_equal(ctx.decode_stream(data, [len(toks)])[0], toks)
    assert (bits[0] - orc.ideal_bits) / len(toks) < 0.01


def test_backward_at_full_vocabulary_64_rows(dev):
    """The differentiation workload's own size: V = 49,152 and 64 rows (one per stream of the
    batch), five experts.  GPU gradients against the oracle's closed form, norm-wise 1e-4 and per
    element (relative 1e-4 with an absolute floor of 1e-10), and against central finite
    differences of the oracle loss (h = 1e-4, FP64), summed row by row so that the cancellation
    of each difference stays at the rounding of one row's loss."""
    from paper_2602_19626_amd.ensemble import ensemble_loss
    z, b, theta, P, t = _case(11, rows=64, v=49152)
    tz = torch.tensor(z, dtype=torch.float32, device=dev)
    tb = torch.tensor(b, dtype=torch.float32, device=dev, requires_grad=True)
    tth = torch.tensor(theta, dtype=torch.float32, device=dev, requires_grad=True)
    tP = torch.tensor(P, dtype=torch.float32, device=dev).contiguous()
    tt = torch.tensor(t, dtype=torch.int32, device=dev)
    loss = ensemble_loss(tz, tb, tth, tP, tt)
    loss.sum().backward()
    gb = tb.grad.double().cpu().numpy()
    gth = tth.grad.double().cpu().numpy()
    z32, b32, th32, P32 = (np.float64(np.float32(x)) for x in (z, b, theta, P))
    ref_loss, ref_gb, ref_gth = _oracle_grads(z32, b32, th32, P32, t)
    assert abs(float(loss.detach().sum()) - ref_loss) / abs(ref_loss) < 1e-5
    assert np.linalg.norm(gb - ref_gb) / np.linalg.norm(ref_gb) < 1e-4
    assert np.linalg.norm(gth - ref_gth) / np.linalg.norm(ref_gth) < 1e-4
    assert np.all(np.abs(gb - ref_gb) <= 1e-4 * np.abs(ref_gb) + 1e-10)
    assert np.all(np.abs(gth - ref_gth) <= 1e-4 * np.abs(ref_gth) + 1e-10)

    h = 1e-4
    rows = range(z.shape[0])

    def fd(th_p, b_p, th_m, b_m):
        return sum((EnsembleGate.loss(th_p, b_p, z32[r], list(P32[r]), int(t[r]))
                    - EnsembleGate.loss(th_m, b_m, z32[r], list(P32[r]), int(t[r]))) / (2 * h)
                   for r in rows)

    fd_th = np.array([fd(th32 + h * e, b32, th32 - h * e, b32) for e in np.eye(len(theta))])
    assert np.linalg.norm(gth - fd_th) / np.linalg.norm(fd_th) < 1e-4
    idx = np.unique(np.concatenate([t[:12], np.arange(0, z.shape[1], 4099)]))
    fd_b = []
    for i in idx:
        e = np.zeros_like(b32)
        e[i] = h
        fd_b.append(fd(th32, b32 + e, th32, b32 - e))
    fd_b = np.array(fd_b)
    assert np.linalg.norm(gb[idx] - fd_b) / np.linalg.norm(fd_b) < 1e-4
    assert np.all(np.abs(gb[idx] - fd_b) <= 1e-4 * np.abs(fd_b) + 1e-9)
