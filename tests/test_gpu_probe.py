"""The streaming-ceiling probe kernel moves exactly the bytes it claims: a
copy reproduces its source in every split, unroll and cache-policy form
(including a ragged tail), the write-only stream writes its pattern
everywhere, and the read-only stream reads every vector once.  Invalid
requests are refused on the host."""
import pytest

from paper_0712_0813_amd import ce

pytestmark = pytest.mark.gpu

# 16-byte vectors per part: not a multiple of any block's span (256 x unroll)
PER = 256 * 8 * 3 + 37


@pytest.mark.parametrize("parts", [1, 4])
@pytest.mark.parametrize("unroll", [1, 8])
@pytest.mark.parametrize("nt", [0, 3])
def test_copy_reproduces_source(parts, unroll, nt):
    import torch
    n = PER * parts * 4  # float32 elements
    x = torch.randint(-2 ** 20, 2 ** 20, (n,), dtype=torch.int32, device="cuda").float()
    y = torch.zeros_like(x)
    ms = ce.ce_stream_probe(ce.CE_PROBE_COPY, x.data_ptr(), y.data_ptr(), 4 * n, parts=parts, unroll=unroll,
                            nt=nt, grid=7, reps=2)
    torch.cuda.synchronize()
    assert ms > 0 and torch.equal(x, y)


@pytest.mark.parametrize("parts", [1, 4])
def test_write_and_read_streams(parts):
    import torch
    n = PER * parts * 4
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    ce.ce_stream_probe(ce.CE_PROBE_WRITE, None, y.data_ptr(), 4 * n, parts=parts, unroll=4, nt=2, grid=5, reps=1)
    torch.cuda.synchronize()
    pattern = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").repeat(n // 4)
    assert torch.equal(y, pattern)
    # read-only: every thread sums the vectors it loads into dst; with all
    # ones the sums are exact small integers and add up to the vector count
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    grid = 6
    d = torch.full((grid * 256 * 4,), -1.0, dtype=torch.float32, device="cuda")
    ce.ce_stream_probe(ce.CE_PROBE_READ, x.data_ptr(), d.data_ptr(), 4 * n, parts=parts, unroll=2, nt=1,
                       grid=grid, reps=1)
    torch.cuda.synchronize()
    sums = d.view(-1, 4)
    assert torch.equal(sums[:, 0], sums[:, 3]) and float(sums[:, 0].sum()) == PER * parts


def test_invalid_requests_are_refused():
    import torch
    x = torch.zeros(4096, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    bad = [dict(parts=3), dict(unroll=3), dict(nt=4), dict(grid=-1)]
    for kw in bad:
        with pytest.raises(ce.CeError) as ei:
            ce.ce_stream_probe(ce.CE_PROBE_COPY, x.data_ptr(), y.data_ptr(), 4 * 4096, **kw)
        assert ei.value.status == ce.CE_EINVAL, kw
    with pytest.raises(ce.CeError):   # not a multiple of 16 x parts
        ce.ce_stream_probe(ce.CE_PROBE_COPY, x.data_ptr(), y.data_ptr(), 4 * 4096 - 16, parts=4)
    with pytest.raises(ce.CeError):   # misaligned
        ce.ce_stream_probe(ce.CE_PROBE_COPY, x.data_ptr() + 4, y.data_ptr(), 1024)
    with pytest.raises(ce.CeError):   # read sums would not fit in dst (grid x 256 vectors > bytes)
        ce.ce_stream_probe(ce.CE_PROBE_READ, x.data_ptr(), y.data_ptr(), 4 * 4096, grid=8)
    with pytest.raises(ce.CeError):
        ce.ce_stream_probe(7, x.data_ptr(), y.data_ptr(), 4 * 4096)
