"""Write the stored oracle values (calls only oracle/).

    python tests/golden/make_golden.py            # both files
    python tests/golden/make_golden.py small      # only the 4^3 sweep

oracle_trajectory_4cubed.json: 4^3 periodic lattice, M = 256, Jackson kernel,
beta = 20, mu = 0, uniform-sphere starts and proposals, Philox key (1, 0): the
first 64 proposals (one sweep) with the oracle's own Metropolis decisions.

oracle_dseff_64cubed.json: 64^3, M = 4096, beta = 20, mu = 0, uniform-sphere
starts and proposals, Philox key (11, 0): the first two proposals (the
oracle needs minutes for each, too long to run inside a GPU test).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def trajectory():
    m = oracle.Model(L=4, M=256, beta=20.0, seed=1, chain_id=0)
    th, ph = oracle.init_spins(m, 0)
    out = []
    for idx in range(m.N):
        r = oracle.step(m, th, ph, idx)
        out.append({"index": r.index, "site": r.site, "theta_new": r.theta_new,
                    "phi_new": r.phi_new, "u": r.u, "dseff": r.dseff,
                    "accepted": r.accepted})
    return {"lattice": 4, "M": 256, "beta": 20.0, "mu": 0.0, "seed": 1, "chain_id": 0,
            "kernel": "jackson", "proposals": out,
            "magnetization": oracle.magnetization(4, th, ph)}


def large():
    m = oracle.Model(L=64, M=4096, beta=20.0, seed=11, chain_id=0)
    th, ph = oracle.init_spins(m, 0)
    out = []
    for idx in range(2):
        r = oracle.step(m, th, ph, idx)
        out.append({"index": r.index, "site": r.site, "theta_new": r.theta_new,
                    "phi_new": r.phi_new, "u": r.u, "dseff": r.dseff,
                    "accepted": r.accepted, "phase_top": r.phase_top})
    return {"lattice": 64, "M": 4096, "beta": 20.0, "mu": 0.0, "seed": 11, "chain_id": 0,
            "kernel": "jackson", "proposals": out}


if __name__ == "__main__":
    path = os.path.join(HERE, "oracle_trajectory_4cubed.json")
    with open(path, "w") as f:
        json.dump(trajectory(), f, indent=1)
    print(path)
    if len(sys.argv) < 2 or sys.argv[1] != "small":
        path = os.path.join(HERE, "oracle_dseff_64cubed.json")
        with open(path, "w") as f:
            json.dump(large(), f, indent=1)
        print(path)
