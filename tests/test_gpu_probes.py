"""The peak-rate probes (sb_peak_probe) compute exactly what their closed forms say, so the rates the
bench derives from them rest on known work: FP32 FMA chains bit for bit against a host emulation of
one rounding per step, LDS sums bit for bit against the same reads summed on the host in the kernel's
order, and the copy bitwise."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = 256


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sb(torch):
    from paper_2504_08081_amd import saltbf
    saltbf.lib()
    return saltbf


def fma_chains_host(iters):
    """Sum of the 16 chains x <- fma(x, a, b), chain j from j, each step rounded once to float32 (a x + b
    is exact in float64 here: x has 24 significant bits, a 10, b is a power of two)."""
    a, b = 1023.0 / 1024.0, 1.0 / 1024.0
    s = np.float32(0.0)
    for j in range(16):
        x = np.float32(j)
        for _ in range(iters):
            x = np.float32(float(x) * a + b)
        s = np.float32(s + x)
    return s


def test_fma_probe_matches_its_closed_form(sb, torch):
    n, iters = 3, 37
    dst = torch.full((n * THREADS,), -1.0, device="cuda")
    work = sb.peak_probe(sb.SB_PROBE_FMA_F32, n, iters, dst=dst)
    torch.cuda.synchronize()
    assert work == 2.0 * n * THREADS * 16 * iters
    got = dst.cpu().numpy()
    assert np.all(got == fma_chains_host(iters)), (got[:4], fma_chains_host(iters))


def test_lds_probe_reads_every_entry_it_claims(sb, torch):
    n, iters = 2, 5
    dst = torch.full((n * THREADS,), -1.0, device="cuda")
    work = sb.peak_probe(sb.SB_PROBE_LDS_READ, n, iters, dst=dst)
    torch.cuda.synchronize()
    assert work == float(n * iters * 16384)
    t = np.arange(THREADS)
    acc = np.zeros((4, THREADS), np.float32)
    for k in range(iters):
        for r in range(4):
            i = ((t ^ (k & 255)) + 256 * r).astype(np.float32)
            for c, off in enumerate((0.0, 0.25, 0.5, 0.75)):
                acc[c] = acc[c] + (i + np.float32(off))
    want = (acc[0] + acc[1]) + (acc[2] + acc[3])
    got = dst.cpu().numpy().reshape(n, THREADS)
    assert np.array_equal(got[0], want) and np.array_equal(got[1], want)


def test_copy_probe_is_a_copy(sb, torch):
    nbytes = (1 << 20) + 48                      # several grid strides and a ragged tail
    g = torch.Generator(device="cpu").manual_seed(5)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (nbytes // 4,), dtype=torch.int32, generator=g).cuda()
    dst = torch.zeros_like(src)
    work = sb.peak_probe(sb.SB_PROBE_COPY, nbytes, src=src, dst=dst)
    torch.cuda.synchronize()
    assert work == 2.0 * nbytes
    assert torch.equal(src, dst)
