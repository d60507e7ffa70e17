"""Writes workloads/rule_s.json: calibrated (C0, s) for rule S per (M, X).

Test infrastructure only (see ``oracle/__init__``). Run from the repository
root: ``python -m oracle.calibrate_rule_s``. X is the half-width of the master
grid in cells (a power of two at least as large as the workload's), s is in
inverse cells (grid units, h = 1); a workload with cell size h uses s/h.
The fit minimises the entrywise maximum relative error of the rank-(M+1) tensor
against the exact Galerkin tensor (reading G2 of the quadrature).
"""
import json
import os

from .quadrature import calibrate_rule_s

MS = (29, 35, 41, 47, 53, 59)
XS = (256, 512, 1024, 2048, 4096, 8192, 16384)


def main():
    table = []
    for X in XS:
        for M in MS:
            C0, s, err = calibrate_rule_s(M, X)
            table.append({"M": M, "X": X, "C0": C0, "s": s, "max_rel_err": err})
            print(f"M={M:3d} X={X:6d} C0={C0:.6f} s={s:.6e} err={err:.3e}", flush=True)
    path = os.path.join(os.path.dirname(__file__), "..", "workloads", "rule_s.json")
    with open(path, "w") as f:
        json.dump({"grid_units": True, "note": "written by oracle/calibrate_rule_s.py",
                   "table": table}, f, indent=1)


if __name__ == "__main__":
    main()
