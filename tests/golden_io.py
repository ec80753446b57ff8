"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _mat(text):
    rows = [r.split() for r in text.split(";")]
    return np.array([[int(x) for x in r] for r in rows], dtype=np.uint32)


def hand_examples():
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, "hand_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("case"):
                cur = {"k": None}
                for kv in line.split()[1:]:
                    key, val = kv.split("=")
                    cur[key] = int(val)
                cases.append(cur)
            else:
                tag, rest = line.split(None, 1)
                cur[tag] = _mat(rest)
    for c in cases:
        if c.get("k") == 0:
            m, n = c["C"].shape
            c["A"] = np.zeros((m, 0), dtype=np.uint32)
            c["B"] = np.zeros((0, n), dtype=np.uint32)
    return cases


def winolevel():
    table = {}
    with open(os.path.join(GOLDEN, "winolevel.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            n = int(parts[0])
            vals = [int(x.rstrip("*")) for x in parts[1:]]
            best = [i for i, x in enumerate(parts[1:]) if x.endswith("*")][0]
            table[n] = (vals, best)
    return table


def trsm_params():
    rows = []
    with open(os.path.join(GOLDEN, "trsm_params.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(tuple(int(x) for x in line.split()))
    return rows


def lqup_hand():
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, "lqup_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("case"):
                cur = {}
                for kv in line.split()[1:]:
                    key, val = kv.split("=")
                    cur[key] = int(val)
                cases.append(cur)
                continue
            tag, rest = line.split(None, 1)
            if tag in ("A", "F"):
                cur[tag] = _mat(rest)
            elif tag in ("pivrows", "colperm"):
                cur[tag] = [int(x) for x in rest.split()]
            else:
                cur[tag] = int(rest)
    return cases
