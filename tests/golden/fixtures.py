"""Readers for the small text fixtures in this folder (each file cites its source)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read_kv(name):
    out = {}
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()[:2]
            out[k] = int(v, 0)
    return out


def read_rows(name):
    rows = []
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(tok, 0) for tok in line.split()])
    return rows
