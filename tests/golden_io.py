"""Reader of the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_worked_example(name="worked_example.txt"):
    d = {"A": [], "B": [], "Cin": [], "C": [], "checksums": [], "fault": [], "expect": []}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key in ("A", "B", "Cin", "C"):
                d[key].append([float(v) for v in vals])
            elif key in ("checksums", "fault", "expect"):
                d[key].append(vals)
            else:
                d[key] = float(vals[0])
    for key in ("A", "B", "Cin", "C"):
        d[key] = np.asfortranarray(np.array(d[key]))
    for key in ("m", "n", "k", "tm", "tn", "bk"):
        d[key] = int(d[key])
    return d


def read_threshold_example(name="threshold_example.txt"):
    d = {"A": [], "B": [], "Cin": []}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            if key in d:
                d[key].append([float(v) for v in vals])
            elif len(vals) == 1:
                d[key] = float(vals[0])
            else:
                d[key] = np.array([float(v) for v in vals])
    for key in ("A", "B", "Cin"):
        d[key] = np.asfortranarray(np.array(d[key]))
    return d
