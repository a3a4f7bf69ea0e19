"""Critical-chain walk of the row-timeline tool on a hand-made timeline."""
import numpy as np

from paper_2306_14337_amd import timeline


def test_chain_follows_the_input_that_finished_last():
    # rows 0..5; row 3 depends on 0 and 1, row 4 on 2 and 3, row 5 on 4; row 1
    # finishes after row 0, so the chain runs 1 -> 3 -> 4 -> 5
    deps = {0: [], 1: [], 2: [], 3: [0, 1], 4: [2, 3], 5: [4]}
    rowptr, colind = [0], []
    for i in range(6):
        colind += deps[i] + [i]
        rowptr.append(len(colind))
    rowptr = np.array(rowptr)
    colind = np.array(colind)
    tl = np.array([[0, 0, 10, 2], [0, 0, 30, 2], [0, 0, 50, 2],
                   [5, 30, 40, 3], [6, 50, 70, 3], [60, 70, 90, 3]], dtype=np.int64)
    assert timeline.critical_chain(tl, rowptr, colind) == [2, 4, 5]
    tl[2, 2] = 20  # now row 3 (via row 1) is the later input of row 4
    assert timeline.critical_chain(tl, rowptr, colind) == [1, 3, 4, 5]
    text = timeline.summary(tl, rowptr, colind, c0=6)
    assert "critical chain: 4 rows" in text and "2 links join consecutive rows" in text
    # rows without a record (kind 0) are skipped as inputs
    tl[1, 3] = 0
    assert timeline.critical_chain(tl, rowptr, colind) == [0, 3, 4, 5]


def test_multiply_adds_count_the_pivot_rows_u_entries():
    # row i pays, for each pivot k < min(i, c0) in its L part, one multiply-add
    # per U entry of row k right of k's diagonal; checked against loops over a
    # small dense-pattern factor
    rows = [[0, 2], [1, 3], [0, 2, 3], [1, 2, 3]]
    rowptr = np.cumsum([0] + [len(r) for r in rows])
    colind = np.array([c for r in rows for c in r])
    for c0, want in ((4, [0, 0, 1, 2]), (2, [0, 0, 1, 1]), (0, [0, 0, 0, 0])):
        got = timeline.multiply_adds(rowptr, colind, c0)
        brute = [sum(sum(1 for c in rows[k] if c > k) for k in r if k < i and k < c0)
                 for i, r in enumerate(rows)]
        assert list(got) == want == brute
