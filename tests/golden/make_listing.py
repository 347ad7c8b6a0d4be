#!/usr/bin/env python3
"""Extract the implementation listings of App. A (53- and 54-qubit circuits)
into tab-separated fixtures: one row per listing line, continuation lines
joined, columns as printed (tensor, phase, mode, depth, gate, arguments).

    python tests/golden/make_listing.py /root/reference/PAPER.md

writes tests/golden/listing_53q.txt and tests/golden/listing_54q.txt.  The
values are the paper's own (App. A); nothing is computed here.
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def listings(text: str):
    """The two longtable bodies, in order (53 qubits, then 54)."""
    out = []
    pos = 0
    while True:
        a = text.find("\\begin{longtable}", pos)
        if a < 0:
            return out
        b = text.find("\\end{longtable}", a)
        out.append(text[a:b])
        pos = b


def rows(body: str):
    res = []
    for line in body.splitlines():
        line = line.strip()
        if not line.endswith("\\\\"):
            continue
        parts = [p.strip() for p in line[:-2].split("&")]
        if len(parts) != 6 or parts[0] == "Tensor":
            continue
        if parts[0] == "" and parts[2] == "":          # continuation of the arguments
            res[-1][5] += parts[5].replace("\\quad", "").strip()
            continue
        res.append(parts)
    return res


def main(path: str) -> None:
    text = open(path).read()
    bodies = listings(text)
    assert len(bodies) == 2, "expected the 53- and 54-qubit listings"
    for n, body in zip((53, 54), bodies):
        out = os.path.join(HERE, f"listing_{n}q.txt")
        with open(out, "w") as f:
            f.write(f"# App. A: implementation listing for the {n}-qubit, 20-cycle circuit, as printed\n")
            f.write("# tensor\tphase\tmode\tdepth\tgate\targuments\n")
            for r in rows(body):
                f.write("\t".join(r) + "\n")
        print(f"wrote {out}")


if __name__ == "__main__":
    main(sys.argv[1])
