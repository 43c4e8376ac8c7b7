"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _vid(c):
    return ord(c) - ord("a")


def fig2():
    """(n, src, dst, phi) of the Example 2 graph, edges in file order."""
    src, dst, phi = [], [], []
    with open(os.path.join(GOLDEN, "fig2_example2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b, k = line.split()
            src.append(_vid(a))
            dst.append(_vid(b))
            phi.append(int(k))
    return 12, np.array(src, np.int32), np.array(dst, np.int32), np.array(phi, np.int32)


def example4():
    """List of (quantity, (u, v), vertex-or-None, value)."""
    out = []
    with open(os.path.join(GOLDEN, "example4_bounds.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            u, v = parts[1].split("-")
            vert = _vid(parts[2]) if len(parts) == 4 else None
            out.append((parts[0], (_vid(u), _vid(v)), vert, int(parts[-1])))
    return out


def edge_index(src, dst, u, v):
    for i in range(len(src)):
        if {int(src[i]), int(dst[i])} == {u, v}:
            return i
    raise KeyError((u, v))


def oracle_record(name):
    """Fields of tests/golden/oracle_<name>.txt (written by make_golden.py), or
    None if the file has not been generated."""
    path = os.path.join(GOLDEN, "oracle_%s.txt" % name)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            val = val.strip()
            if key in ("n", "m", "triangles", "kmax", "graphs", "cmax"):
                rec[key] = int(val)
            elif key == "cohesion":
                rec[key] = {a: (float(b) if a.startswith("CC") else int(b))
                            for a, b in (t.split("=") for t in val.split())}
            elif key in ("graph_kmax", "graph_m"):
                rec[key] = [int(t) for t in val.split()]
            elif key == "class_sizes":
                rec[key] = {int(a): int(b) for a, b in (t.split(":") for t in val.split())}
            else:
                rec[key] = val
    return rec


def int32_digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def example3():
    """Example 3's fixture: dict with part (vertex -> 1..3), bound ((u, v) ->
    value), phi2 (list of (u, v)) and classes (k -> list of (u, v)); (u, v)
    with u < v."""
    out = {"part": {}, "bound": {}, "phi2": [], "classes": {}}

    def pair(t):
        a, b = t.split("-")
        u, v = _vid(a), _vid(b)
        return (min(u, v), max(u, v))

    with open(os.path.join(GOLDEN, "example3_bottomup.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "part":
                out["part"][_vid(t[1])] = int(t[2])
            elif t[0] == "bound":
                out["bound"][pair(t[1])] = int(t[2])
            elif t[0] == "phi2":
                out["phi2"].extend(pair(x) for x in t[1:])
            elif t[0] == "class":
                out["classes"][int(t[1])] = [pair(x) for x in t[2:]]
    return out
