"""Readers for the hand-written fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _pairs(tokens):
    out = []
    for t in tokens:
        k, i = t.split(":")
        out.append((int(k), int(i)))
    return out


def stage_cases():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "stages_small.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = {"name": tok[1], "seed": 0}
            elif tok[0] == "end":
                cases.append(cur)
                cur = None
            elif tok[0] == "mode":
                cur["mode"] = 0 if tok[1] == "RANDOM" else 1
            elif tok[0] in ("p", "s", "seed"):
                cur[tok[0]] = int(tok[1])
            elif tok[0] == "keys":
                cur["keys"] = np.array([int(t) for t in tok[1:]], dtype=np.uint32)
            elif tok[0] in ("sample", "splitters"):
                cur[tok[0]] = _pairs(tok[1:])
            elif tok[0] == "counts":
                cur["counts"] = [int(t) for t in tok[1:]]
    return cases


def splitmix64_vectors():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        lines = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    seed = int(lines[0].split()[1])
    return seed, [int(v) for v in lines[1:]]


def lemma1_cases():
    """(n, p, r, safe, tight, final) rows of tests/golden/lemma1.txt."""
    rows = []
    with open(os.path.join(GOLDEN, "lemma1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            rows.append((int(t[0]), int(t[1]), int(t[2]), int(t[3]), int(t[4]), float(t[5])))
    return rows
