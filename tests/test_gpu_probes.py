"""The bandwidth probes move the data they claim: the copies reproduce
their source, the write fills, and each stream mix writes the xor of its
read streams (written stream k: read streams k, k + NW, k + 2 NW, ...), on
sizes with a ragged tail of the grid-stride loop."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_13768_amd import wfa
    wfa.lib()
    return torch, wfa


def _rand_words(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randint(-2**31, 2**31 - 1, (n,), generator=g, dtype=torch.int64).to(torch.int32)


@pytest.mark.parametrize("nbytes", [4096, 16 * 12345, 1 << 22])
@pytest.mark.parametrize("blocks", [0, 3, 64])
def test_copies_and_write(env, nbytes, blocks):
    torch, wfa = env
    src = _rand_words(torch, nbytes // 4, nbytes).cuda()
    for kind in (wfa.PROBE_COPY, wfa.PROBE_COPY_PLAIN, wfa.PROBE_COPY32):
        if kind == wfa.PROBE_COPY32 and nbytes % 32:
            continue
        dst = torch.full_like(src, 7)
        gbps = wfa.bandwidth_probe(kind, src, dst, reps=2, blocks=blocks)
        torch.cuda.synchronize()
        assert gbps > 0 and torch.equal(dst, src), (kind, nbytes, blocks)
    dst = torch.full_like(src, 7)
    assert wfa.bandwidth_probe(wfa.PROBE_WRITE, src, dst, reps=1, blocks=blocks) > 0
    torch.cuda.synchronize()
    assert int(dst.abs().max()) == 0
    assert wfa.bandwidth_probe(wfa.PROBE_READ, src, dst, reps=1, blocks=blocks) > 0


@pytest.mark.parametrize("stream_bytes", [16, 16 * 1001, 1 << 21])
@pytest.mark.parametrize("blocks", [0, 5])
def test_stream_mixes(env, stream_bytes, blocks):
    torch, wfa = env
    for kind in (wfa.PROBE_MIX_6R4W, wfa.PROBE_MIX_3R1W):
        nr, nw = wfa.PROBE_STREAMS[kind]
        n = stream_bytes // 4
        src = _rand_words(torch, nr * n, stream_bytes + kind).cuda()
        dst = torch.full((nw * n,), 7, dtype=torch.int32, device="cuda")
        gbps = wfa.bandwidth_probe(kind, src, dst, reps=1, blocks=blocks)
        torch.cuda.synchronize()
        assert gbps > 0
        s = src.cpu().view(nr, n)
        want = torch.zeros(nw, n, dtype=torch.int32)
        for j in range(nr):
            want[j % nw] ^= s[j]
        assert torch.equal(dst.cpu().view(nw, n), want), (kind, stream_bytes, blocks)
    with pytest.raises(ValueError):
        wfa.bandwidth_probe(wfa.PROBE_MIX_6R4W, torch.empty(64, device="cuda"),
                            torch.empty(64, device="cuda"))
