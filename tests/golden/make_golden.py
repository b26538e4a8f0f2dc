"""Writes the text fixtures in this folder.  It calls only the CPU oracle
and the seeded input generators, never the GPU library.

The paper prints no worked Cholesky example, so the fixtures hold the
oracle's own output on a tiny seeded case; they guard the oracle against
unintended changes and give the GPU tests a stored expectation.

    python -m tests.golden.make_golden
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def case_grid2d_4x4():
    import workloads as W
    return W.small_grid((4, 4), order="nd", seed=2024)


def write_fixture(path, arrays: dict, header: str):
    with open(path, "w") as f:
        for line in header.strip().splitlines():
            f.write("# " + line + "\n")
        for k, v in arrays.items():
            v = np.asarray(v).ravel()
            if v.dtype.kind == "f":
                vals = " ".join(float(t).hex() for t in v)
                f.write("%s f %s\n" % (k, vals))
            else:
                f.write("%s i %s\n" % (k, " ".join(str(int(t)) for t in v)))


def read_fixture(path) -> dict:
    out = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, kind, *vals = line.split()
            if kind == "f":
                out[key] = np.array([float.fromhex(t) for t in vals])
            else:
                out[key] = np.array([int(t) for t in vals], dtype=np.int64)
    return out


def main():
    import oracle
    w = case_grid2d_4x4()
    p = w.pattern
    s = oracle.symbolic(p.n, p.colptr, p.rowind, w.perm)
    Lx, info = oracle.factor(p.n, p.colptr, p.rowind, w.values[0], s)
    assert info == 0
    x = oracle.solve(s, Lx, w.b[0])
    write_fixture(os.path.join(HERE, "grid2d_4x4_nd.txt"), {
        "perm": w.perm, "colptr": p.colptr, "rowind": p.rowind,
        "values": w.values[0], "b": w.b[0], "parent": s.parent,
        "Lcolptr": s.Lcolptr, "Lrowind": s.Lrowind, "Lx": Lx, "x": x,
    }, header="""
4x4 5-point grid, geometric nested dissection, Laplacian value rule, seed 2024.
Written by tests/golden/make_golden.py from the CPU oracle (FP64, up-looking
Cholesky); floats are exact hex.  No value here comes from the GPU library.
""")


if __name__ == "__main__":
    main()
