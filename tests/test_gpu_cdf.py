"""GPU parity of the CDF-24 kernels (section 3.4) against the oracle quantiser: bit-exact on the
same float32 probabilities, including adversarial rows."""
import numpy as np
import pytest

from oracle.cdf import quantize_cdf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
T24 = 1 << 24


@pytest.fixture(scope="module")
def nc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_19626_amd as m
    return m


def _gpu_cdf(nc, rows):
    p = torch.from_numpy(np.ascontiguousarray(rows, dtype=np.float32)).cuda()
    cdf, st = nc.quantize_cdf24(p)
    torch.cuda.synchronize()
    return cdf.cpu().numpy().view(np.uint32), st.cpu().numpy()


def _check(nc, rows):
    cdf, st = _gpu_cdf(nc, rows)
    for r in range(rows.shape[0]):
        assert st[r] == 0, r
        ref = quantize_cdf(rows[r].astype(np.float32))
        assert np.array_equal(cdf[r].astype(np.int64), ref), f"row {r}"


def test_random_full_vocab_rows(nc):
    rng = np.random.default_rng(0)
    rows = np.stack([rng.dirichlet(np.full(49152, a)) for a in (0.01, 0.1, 1.0, 10.0)])
    _check(nc, rows.astype(np.float32))


@pytest.mark.parametrize("n", [16, 64, 65, 80])
def test_full_vocab_both_launch_paths(nc, n):
    """At V = 49,152 up to 64 rows run the segment kernels and more rows the one-workgroup-per-row
    kernel; both must equal the oracle, and a row's CDF must not depend on the batch it is in."""
    rng = np.random.default_rng(100 + n)
    alphas = (0.005, 0.05, 0.5, 5.0)
    rows = np.stack([rng.dirichlet(np.full(49152, alphas[i % 4])) for i in range(n)])
    rows = rows.astype(np.float32)
    rows[n // 2] = 0.0
    rows[n // 2, 12345] = 1.0
    _check(nc, rows)
    head, _ = _gpu_cdf(nc, rows[:16])
    full, _ = _gpu_cdf(nc, rows)
    assert np.array_equal(head, full[:16])


def test_worked_examples(nc):
    rows = np.full((1, 512), 2.0 ** -9, dtype=np.float32)
    cdf, st = _gpu_cdf(nc, rows)
    c = np.diff(cdf[0].astype(np.int64))
    assert st[0] == 0 and c[0] == 33279 and np.all(c[1:] == 32767)
    rows = np.full((1, 49152), 1.0 / 49152, dtype=np.float32)
    cdf, _ = _gpu_cdf(nc, rows)
    c = np.diff(cdf[0].astype(np.int64))
    assert c[0] == 65876 and np.all(c[1:] == 340)
    oh = np.zeros((1, 49152), np.float32)
    oh[0, 40000] = 1.0
    cdf, _ = _gpu_cdf(nc, oh)
    c = np.diff(cdf[0].astype(np.int64))
    assert c[40000] == T24 - 49152 + 1 and cdf[0, -1] == T24


@pytest.mark.parametrize("v", [1, 2, 3, 5, 511, 4095, 4096, 4097, 5000, 12289, 49152, 65536])
def test_ragged_vocab_sizes(nc, v):
    rng = np.random.default_rng(v)
    rows = np.stack([rng.dirichlet(np.full(v, 0.3)) for _ in range(3)]).astype(np.float32)
    _check(nc, rows)


def test_adversarial_rows(nc):
    v = 49152
    rng = np.random.default_rng(1)
    rows = []
    p = rng.dirichlet(np.full(v, 0.05)).astype(np.float32)
    p[[10, 30000]] = p.max()                       # tie for the maximum: lowest index wins
    rows.append(p / np.float32(p.sum()))
    q = rng.dirichlet(np.full(v, 0.5)).astype(np.float32) * np.float32(1.00001)  # sum > 1
    rows.append(q)
    z = np.zeros(v, np.float32)
    z[[0, v - 1]] = 0.5                             # mass at both ends, zeros elsewhere
    rows.append(z)
    s = rng.dirichlet(np.full(v, 0.05)).astype(np.float32)
    s[::7] = np.float32(1e-40)                      # subnormals
    rows.append(s)
    t = np.full(v, np.float32(1.0 / v))
    t[12345] = np.nextafter(t[12345], np.float32(1))  # near-integer products
    rows.append(t)
    _check(nc, np.stack(rows))


def test_invalid_rows_flagged(nc):
    v = 4096
    good = np.full(v, 1.0 / v, np.float32)
    bad = np.stack([good.copy() for _ in range(4)])
    bad[0, 5] = np.nan
    bad[1, 6] = -1e-3
    bad[2, :] = 1.0                                  # mass far above the total
    bad[3, 7] = 1.5
    rows = np.concatenate([good[None], bad])
    _, st = _gpu_cdf(nc, rows)
    assert list(st) == [0, 1, 1, 1, 1]


def test_batch_and_interval_lookup(nc):
    rng = np.random.default_rng(2)
    v = 49152
    rows = np.stack([rng.dirichlet(np.full(v, 0.02)) for _ in range(64)]).astype(np.float32)
    p = torch.from_numpy(rows).cuda()
    cdf, st = nc.quantize_cdf24(p)
    tok = rng.integers(0, v, size=64).astype(np.int32)
    enc = nc.cdf_interval(cdf, torch.from_numpy(tok).cuda(), 0).cpu().numpy()
    c = cdf.cpu().numpy().view(np.uint32).astype(np.int64)
    targets = rng.integers(0, T24, size=64).astype(np.int32)
    dec = nc.cdf_interval(cdf, torch.from_numpy(targets).cuda(), 1).cpu().numpy()
    for r in range(64):
        ref = quantize_cdf(rows[r])
        assert np.array_equal(c[r], ref)
        assert tuple(enc[r]) == (tok[r], ref[tok[r]], ref[tok[r] + 1])
        s = int(np.searchsorted(ref, targets[r], side="right") - 1)
        assert tuple(dec[r].astype(np.int64)) == (s, ref[s], ref[s + 1])


def test_two_streams_do_not_share_a_workspace(nc):
    """Two row sets (both on the segment path, which keeps partials in the workspace) quantised on
    two streams whose work overlaps: each equals the oracle."""
    rng = np.random.default_rng(7)
    a = np.stack([rng.dirichlet(np.full(49152, 0.05)) for _ in range(48)]).astype(np.float32)
    b = np.stack([rng.dirichlet(np.full(49152, 2.0)) for _ in range(40)]).astype(np.float32)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        outs.append((nc.quantize_cdf24(ta, stream=s1), nc.quantize_cdf24(tb, stream=s2)))
    torch.cuda.synchronize()
    for (ca, sa), (cb, sb) in outs:
        ca = ca.cpu().numpy().view(np.uint32)
        cb = cb.cpu().numpy().view(np.uint32)
        assert not sa.cpu().numpy().any() and not sb.cpu().numpy().any()
        for r in range(0, 48, 5):
            assert np.array_equal(ca[r].astype(np.int64), quantize_cdf(a[r])), r
        for r in range(0, 40, 5):
            assert np.array_equal(cb[r].astype(np.int64), quantize_cdf(b[r])), r


def _adversarial(v, rng):
    rows = []
    p = rng.dirichlet(np.full(v, 0.05)).astype(np.float32)
    p[[10, v // 2 + 3]] = p.max()                   # tie for the maximum: lowest index wins
    rows.append(p / np.float32(p.sum()))
    rows.append(rng.dirichlet(np.full(v, 0.5)).astype(np.float32) * np.float32(1.00001))
    z = np.zeros(v, np.float32)
    z[[0, v - 1]] = 0.5
    rows.append(z)
    s = rng.dirichlet(np.full(v, 0.05)).astype(np.float32)
    s[::7] = np.float32(1e-40)
    rows.append(s)
    t = np.full(v, np.float32(1.0 / v))
    t[v // 3] = np.nextafter(t[v // 3], np.float32(1))
    rows.append(t)
    oh = np.zeros(v, np.float32)
    oh[v - 2] = 1.0
    rows.append(oh)
    return rows


@pytest.mark.parametrize("v", [512, 2048, 4100, 12288, 49148, 49152])
def test_row_kernel_path_adversarial_and_ragged(nc, v):
    """More than 64 rows of a vocabulary that is a multiple of 4 run the one-workgroup-per-row
    kernel: adversarial rows (ties, mass above one, subnormals, near-integer products, one-hot)
    and random rows, bit-exact with the oracle; invalid rows are flagged."""
    rng = np.random.default_rng(v)
    rows = _adversarial(v, rng)
    while len(rows) < 70:
        rows.append(rng.dirichlet(np.full(v, rng.choice([0.01, 0.3, 3.0]))).astype(np.float32))
    rows = np.stack(rows)
    _check(nc, rows)
    bad = rows.copy()
    bad[3, 5] = np.nan
    bad[40, 6] = -1e-3
    bad[69, :] = 1.0
    _, st = _gpu_cdf(nc, bad)
    assert [r for r in range(70) if st[r]] == [3, 40, 69]
