"""Readers for the text fixtures in this folder (paper worked examples)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _ints(field):
    field = field.strip()
    return [int(x) for x in field.split(",")] if field else []


def paper_examples():
    out = []
    with open(os.path.join(HERE, "paper_examples.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, M, J, expected, cite = [x.strip() for x in line.split("|")]
            out.append(dict(kind=kind, M=int(M), J=_ints(J), expected=_ints(expected), cite=cite))
    return out


def printed_matrix():
    """Entries of 2^8 F^{-1}(I, J) for J = {84, 305, 725, 992}, N = 2^10."""
    rows = []
    with open(os.path.join(HERE, "hidft_matrix_84_305_725_992.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            i, j, re, im = [x.strip() for x in line.split("|")]
            rows.append((int(i), int(j), complex(float(re), float(im))))
    return rows


def part_homogeneous_examples():
    out = []
    with open(os.path.join(HERE, "part_homogeneous_examples.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            M, J, r, level, nodes, cite = [x.strip() for x in line.split("|")]
            groups = [sorted(int(x) for x in g.split(",")) for g in nodes.split(";")]
            out.append(dict(M=int(M), J=_ints(J), r=_ints(r), level=int(level),
                            nodes=sorted(groups), cite=cite))
    return out
