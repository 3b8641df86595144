"""Host-side pieces of the serving loop (no GPU): the packed request layout."""
import numpy as np

from paper_2606_14480_amd import events as ev
from paper_2606_14480_amd import serving


def test_layout_is_aligned_and_disjoint():
    for dims in ((1, 10, 3), (7, 12345, 777), (0, 0, 0), (1000, 1556014, 126295)):
        off, total = serving.layout(*dims)
        spans = sorted((o, o + 4 * n) for o, n in off.values())
        for (a0, a1), (b0, _) in zip(spans, spans[1:]):
            assert a1 <= b0
        assert all(o % 256 == 0 for o, _ in off.values())
        assert spans[-1][1] <= total


def test_pack_round_trip():
    b = ev.generate(ev.config(2, n_events=3))
    off, total = serving.layout(b.n_events, b.n_hits, b.n_velo)
    buf = np.zeros(total, np.uint8)
    serving._pack_into(b, buf, off)
    for f in serving._FIELDS:
        a = np.ascontiguousarray(getattr(b, f))
        o, n = off[f]
        assert n == len(a)
        assert buf[o:o + 4 * n].view(a.dtype).tolist() == a.tolist()
