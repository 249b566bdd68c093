"""Writes the stored expected values under tests/golden/ using only oracle/.

Run from the repository root:  python tests/golden/make_golden.py
It records
  * the seed scan that fixes the 8-qubit all-to-all instance: the first seed
    >= 1002 whose s = 1 Ising ground state is non-degenerate (so the
    "ground-state population" of Sec. V is that of a single level);
  * the split-step FP64 AME ground-state population of that instance on its
    2000-point grid (a2a8_ame_pgs.json), the reference for the stated error
    of the GPU trajectory averages (python tests/golden/make_golden.py --ame);
  * the same for the 4-qubit ring workload (small_ame_pgs.json, --ame-small).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import model  # noqa: E402


def scan_a2a8(start=1002, stop=1100):
    rows = []
    for seed in range(start, stop):
        inst = workloads.pm1_all_to_all(8, seed)
        e = np.sort(model.hz_diag(inst.h, inst.J))
        unique = bool(e[1] - e[0] > 0.5)
        rows.append({"seed": seed, "e0": float(e[0]), "e1": float(e[1]), "unique": unique})
        if unique:
            break
    return rows


def ame_a2a8():
    from oracle import ame, spectrum
    inst = workloads.config_a2a8(10)
    P = ame.split_step(spectrum.table_stream(inst), inst)
    with open(os.path.join(HERE, "a2a8_ame_pgs.json"), "w") as f:
        json.dump({"source": "oracle.ame.split_step over oracle.spectrum.table_stream(workloads.config_a2a8())",
                   "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f,
                   "pgs": [float(p) for p in P]}, f)


def ame_small():
    from oracle import ame, spectrum
    inst = workloads.config_small()
    P = ame.split_step(spectrum.table_stream(inst), inst)
    with open(os.path.join(HERE, "small_ame_pgs.json"), "w") as f:
        json.dump({"source": "oracle.ame.split_step over oracle.spectrum.table_stream(workloads.config_small())",
                   "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f,
                   "pgs": [float(p) for p in P]}, f)


if __name__ == "__main__":
    if "--ame" in sys.argv:
        ame_a2a8()
        sys.exit(0)
    if "--ame-small" in sys.argv:
        ame_small()
        sys.exit(0)
    rows = scan_a2a8()
    with open(os.path.join(HERE, "a2a8_seed_scan.json"), "w") as f:
        json.dump({"source": "oracle.model.hz_diag over workloads.pm1_all_to_all(8, seed)",
                   "rows": rows, "chosen": rows[-1]["seed"]}, f, indent=1)
    print("chosen seed", rows[-1]["seed"])
