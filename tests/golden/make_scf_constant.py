"""Writes the pairing constant g used by the SCF tests (oracle arithmetic only).

g makes the uniform two-species gas on a 64x64 lattice at mu = 1, U = 0 carry
Delta = 0.3 through the zero-temperature gap equation of eq. (densities2):
    1 = g N^-2 sum_{0 < E_k < Ec} 1 / (2 E_k).
"""
import json
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.scf import uniform_densities  # noqa: E402

n, nu = uniform_densities((64, 64), 0.0, 0.3, 1.0, math.pi ** 2 / 2)
g = 0.3 / nu
out = {"source": "tests/golden/make_scf_constant.py (oracle.scf.uniform_densities)",
       "lattice": [64, 64], "mu": 1.0, "Delta": 0.3, "Ec": math.pi ** 2 / 2,
       "g": g, "n_uniform": n}
json.dump(out, open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "scf_constant.json"), "w"),
          indent=1)
print(out)
