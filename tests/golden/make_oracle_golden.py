"""Write oracle_c2_full.json: the oracle's ATM energies for the sc/fcc/bcc
lattices at unit density on the full 263424-node plan.  Calls only oracle/."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    spec = dict(W.SPEC_FULL_3D)
    out = {"spec": spec, "nodes_per_lattice": W.n_nodes(3, spec), "atm": {}, "zetas": {},
           "cite": "oracle (oracle/ezo.c) at the plan above; ATM per Sec. 2, Proposition"}
    for name, A in W.c2_lattices().items():
        t = time.time()
        E, z = oracle.atm(A, spec, zetas=True)
        out["atm"][name] = E
        out["zetas"][name] = {"333": z[0], "m155": z[1], "135": z[2]}
        print(name, E, z, "%.1fs" % (time.time() - t), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c2_full.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
