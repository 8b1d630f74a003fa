"""Writes workloads/codes.json: the exponents of every GB code used here.

The fixed codes are those named in the workload definitions; the random ones
(weight-w pairs "drawn from seed s") are drawn by oracle.codes.draw_gb, this
project's reading of that procedure (redraw until k >= 2).  Calls only the
oracle.  Run from the repository root:  python -m workloads.make_codes
"""
import json
import os

from oracle import codes

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = {
        "G63": dict(l=63, a=list(codes.G63["a"]), b=list(codes.G63["b"])),
        "G127": dict(l=127, a=list(codes.G127["a"]), b=list(codes.G127["b"])),
    }
    for name, l, w, seed in (("G255w3", 255, 3, 7), ("G255w4", 255, 4, 8), ("G511w5", 511, 5, 9)):
        a, b, k, draws = codes.draw_gb(l, w, seed)
        out[name] = dict(l=l, a=list(a), b=list(b), weight=w, seed=seed, draws=draws)
    for name, c in out.items():
        hx, hz = codes.gb_matrices(c["l"], c["a"], c["b"])
        c["k"] = codes.dimension(hx, hz)
        print(name, c)
    with open(os.path.join(HERE, "codes.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
