"""Critical chain of one refactorization from its row timeline.

A handle created with debug_timeline=1 records, for every row its two band
kernels take, when the row started, the last poll that still found one of its
inputs missing, and when its stores completed (kkt_debug_timeline).  Walking
back from the row that finished last, always to the input row that finished
last, gives the chain that set the refactorization's length; each link's
advance (end of the row minus end of its input) splits that length by kernel
kind, and a row that started after its input had already finished shows a
late fetch rather than a slow link.

    python -m paper_2306_14337_amd.timeline --buses 70000

prints a markdown summary for the synthetic system of that size.
"""
from __future__ import annotations

import argparse

import numpy as np

KINDS = {1: "micro rows (one per lane)", 2: "short-row list kernel", 3: "long-row kernel"}


def critical_chain(tl: np.ndarray, rowptr: np.ndarray, colind: np.ndarray) -> list[int]:
    """Rows of the chain ending at the last-finishing recorded row, in order."""
    n = len(rowptr) - 1
    rec = tl[:, 3] > 0
    end = np.where(rec, tl[:, 2], -1)
    i = int(np.argmax(end))
    chain = [i]
    while True:
        cols = colind[rowptr[i]:rowptr[i + 1]]
        deps = cols[(cols < i)]
        deps = deps[rec[deps]] if len(deps) else deps
        if len(deps) == 0:
            break
        i = int(deps[np.argmax(end[deps])])
        chain.append(i)
        if len(chain) > n:
            raise RuntimeError("timeline chain does not terminate")
    return chain[::-1]


def multiply_adds(rowptr: np.ndarray, colind: np.ndarray, c0: int) -> np.ndarray:
    """Per row i: the multiply-adds its sparse pivots cost (for each pivot k
    < min(i, c0) of row i, the U entries of row k right of its diagonal)."""
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    diag = np.full(n, -1, np.int64)
    on = colind == rows
    diag[rows[on]] = np.nonzero(on)[0]
    ulen = np.asarray(rowptr[1:], np.int64) - diag - 1
    piv = (colind < rows) & (colind < c0)
    return np.bincount(rows[piv], weights=ulen[colind[piv]], minlength=n)


def summary(tl: np.ndarray, rowptr: np.ndarray, colind: np.ndarray, c0: int) -> str:
    rec = tl[:, 3] > 0
    chain = critical_chain(tl, rowptr, colind)
    us = tl[:, :3] * 1e-3
    lines = [f"rows recorded: {int(rec.sum())} of {len(tl)}", ""]
    lines += ["| kernel | rows | first start µs | last end µs | median µs from last missing input to end |",
              "|---|---|---|---|---|"]
    for k, name in KINDS.items():
        m = tl[:, 3] == k
        if m.any():
            lines.append(f"| {name} | {int(m.sum())} | {us[m, 0].min():.1f} | {us[m, 2].max():.1f} | "
                         f"{np.median(us[m, 2] - us[m, 1]):.2f} |")
    madd = multiply_adds(rowptr, colind, c0)
    lines += ["", "| kernel | rows | multiply-adds |", "|---|---|---|"]
    for name, m in (("short-row band kernel (micro rows and list)", (tl[:, 3] == 1) | (tl[:, 3] == 2)),
                    ("long-row band kernel", tl[:, 3] == 3)):
        lines.append(f"| {name} | {int(m.sum())} | {int(madd[m].sum())} |")
    adv = np.array([us[b, 2] - us[a, 2] for a, b in zip(chain[:-1], chain[1:])])
    late = np.array([us[b, 0] - us[a, 2] for a, b in zip(chain[:-1], chain[1:])])
    kinds = np.array([tl[b, 3] for b in chain[1:]])
    pos = np.array(chain[1:])
    consec = int(sum(1 for a, b in zip(chain[:-1], chain[1:]) if b == a + 1))
    lines += ["", f"critical chain: {len(chain)} rows, ends at {us[chain[-1], 2]:.1f} µs; "
              f"{consec} links join consecutive rows", "",
              "| links into | links | advance µs (sum) | median µs | p90 µs | fetched after the input ended |",
              "|---|---|---|---|---|---|"]
    groups = [(KINDS[k], kinds == k) for k in (1, 2)]
    groups += [("long-row kernel, rows before the dense block", (kinds == 3) & (pos < c0)),
               ("long-row kernel, dense-block rows (their sparse pivots)", (kinds == 3) & (pos >= c0))]
    for name, m in groups:
        if m.any():
            lines.append(f"| {name} | {int(m.sum())} | {adv[m].sum():.1f} | {np.median(adv[m]):.2f} | "
                         f"{np.percentile(adv[m], 90):.2f} | {int((late[m] > 0).sum())} "
                         f"(late by {np.clip(late[m], 0, None).sum():.1f} µs in all) |")
    return "\n".join(lines)


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--buses", type=int, default=70000)
    ap.add_argument("--seed", type=int, default=103)
    args = ap.parse_args()
    import torch

    from . import binding, kktgen

    pat, seq = kktgen.make_sequence(args.buses, args.seed, 3)
    s = binding.KKTSolver(debug_timeline=1)
    s.analyze(pat.n, pat.rowptr, pat.colind, seq[0][0])
    dev = torch.device("cuda:0")
    for vals, _ in seq:
        s.refactor(torch.from_numpy(vals).to(dev))
    tl = s.debug_timeline()
    rp, ci, _ = s.lu(values=False)
    c0 = pat.n - int(s.info().dense_tail)
    print(f"# Row timeline of one refactorization, B={args.buses} buses (n={pat.n}, "
          f"dense block {s.info().dense_tail})\n")
    print(summary(tl, rp, ci, c0))


if __name__ == "__main__":
    main()
