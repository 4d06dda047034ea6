"""The balanced partition of Alg. 1 (Sec. 4) and the mesh sizes of Tab. 2
(Sec. 5.1), on the host."""
import itertools
import json
import os

import pytest

from paper_2003_08746_amd import partition as P

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("total,nparts", [(1, 1), (7, 1), (7, 7), (7, 3), (361, 8), (1024, 40), (1700, 200),
                                          (5, 8), (0, 3), (128, 6)])
def test_alg1_properties(total, nparts):
    """Sizes sum to the total, differ by at most one, and the larger ones
    are the first (total mod nparts) parts; together these fix the split."""
    s = P.part_sizes(total, nparts)
    assert len(s) == nparts and sum(s) == total
    assert max(s) - min(s) <= 1
    r = total % nparts
    assert all(x == total // nparts + 1 for x in s[:r]) and all(x == total // nparts for x in s[r:])
    off = P.part_offsets(total, nparts)
    assert off[0] == 0 and all(off[p + 1] == off[p] + s[p] for p in range(nparts - 1))


def test_alg1_brute_force():
    """Against the definition by enumeration on tiny cases: among all ways to
    cut [0, total) into nparts contiguous parts, the sizes of Alg. 1 are the
    only ones that differ by at most one with the larger parts first."""
    for total in range(0, 9):
        for nparts in range(1, 6):
            found = []
            for cuts in itertools.combinations_with_replacement(range(total + 1), nparts - 1):
                b = (0,) + cuts + (total,)
                sizes = [b[p + 1] - b[p] for p in range(nparts)]
                if max(sizes) - min(sizes) <= 1 and sizes == sorted(sizes, reverse=True):
                    found.append(sizes)
            assert found == [P.part_sizes(total, nparts)], (total, nparts, found)


def test_block_shape_and_errors():
    assert P.block_shape((1024, 512, 361), (8, 1, 1), (0, 0, 0)) == (128, 512, 361)
    assert P.block_shape((1700, 1700, 361), (3, 2, 1), (0, 1, 0)) == (567, 850, 361)
    assert P.block_shape((1700, 1700, 361), (3, 2, 1), (2, 1, 0)) == (566, 850, 361)
    for bad in ((10, 0, 0), (10, 3, 3), (10, 3, -1), (-1, 2, 0)):
        with pytest.raises(ValueError):
            P.part_size(*bad)


def _quoted(q):
    return float(q[:-1]) * (1e6 if q.endswith("M") else 1e9)


def test_tab2_totals():
    """Each total of Tab. 2 is axial x radial x 361 to the quoted digits,
    and the totals double from mesh to mesh (A to H)."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_meshes.json")))
    naz = g["azimuthal_points"]["value"]
    prev = None
    for m in g["meshes"]:
        n = m["axial"] * m["radial"] * naz
        q = m["total_quoted"]
        digits = len(q[:-1].split(".")[1]) if "." in q else 0
        unit = 1e6 if q.endswith("M") else 1e9
        assert round(n / unit, digits) == _quoted(q) / unit, (m["name"], n, q)
        if prev is not None and m["name"] != "I":
            assert n == 2 * prev
        prev = n
