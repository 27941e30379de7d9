"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_edge_fixture(name):
    edges, rds = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "edge":
                edges.append((int(tok[1]), int(tok[2])))
            elif tok[0] == "rd":
                rds.append((int(tok[1]), int(tok[2]), float(tok[3])))
    return edges, rds
