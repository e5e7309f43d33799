"""The FFT split table survives a process: splits loaded from a file change
the plans built afterwards (seen in hank_plan_block), are written back
unchanged by hank_autotune_save, and malformed files are rejected without
installing anything.  Host only (no GPU)."""
import pytest

import paper_1501_01652_amd as hank


def _split(N):
    b = hank.plan_block("dht0", N, 1e-8, 0, prefer_far=1)
    return b["fft_len"], b["fft_l1"], b["fft_l2"]


def test_autotune_table_roundtrip(tmp_path):
    hank.autotune_reset()
    N = 1 << 18
    L, l1, l2 = _split(N)
    lg = L.bit_length() - 1
    assert l1 * l2 == L
    other = (l2.bit_length() - 1) + 1  # a different supported split: longer columns
    assert 2 * other <= lg
    f = tmp_path / "splits.txt"
    f.write_text("# tuned\n%d %d\n" % (lg, other))
    try:
        hank.autotune_load(str(f))
        L2_, l1b, l2b = _split(N)
        assert L2_ == L and l2b == 1 << other and l1b * l2b == L
        g = tmp_path / "saved.txt"
        hank.autotune_save(str(g))
        lines = [ln.split() for ln in g.read_text().splitlines() if ln and not ln.startswith("#")]
        assert [lg, other] in [[int(a), int(b)] for a, b in lines]
        # a bad line: rejected, nothing installed
        hank.autotune_reset()
        bad = tmp_path / "bad.txt"
        bad.write_text("%d %d\n%d %d\n" % (lg, other, lg, lg))
        with pytest.raises(hank.HankError) as ei:
            hank.autotune_load(str(bad))
        assert ei.value.status == 1
        assert _split(N) == (L, l1, l2)
        with pytest.raises(hank.HankError):
            hank.autotune_load(str(tmp_path / "missing.txt"))
        # the saved file installs the same table again
        hank.autotune_load(str(g))
        assert _split(N)[2] == 1 << other
    finally:
        hank.autotune_reset()
