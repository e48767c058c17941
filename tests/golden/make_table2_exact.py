"""Write table2_exact_rmse.json: the RMSE against the truth of the exact
posterior mean (the oracle's sparse direct solve) for the Table 2 problems,
the Table 1 generator's 128^2, 256^2 and 512^2 grids at 5 % observed, three
truths each.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_table2_exact.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2404_12968_amd import inputs as I  # noqa: E402

SIZES = (128, 256, 512)
TRUTHS = 3


def main():
    out = {"note": "RMSE of the exact posterior mean (sparse LU of the oracle's assembled "
                   "system) against the truth, inputs.table1(n, 0.05, instance)",
           "rmse_exact": {}}
    for n in SIZES:
        vals = []
        for inst in range(TRUTHS):
            p = I.table1(n, 0.05, inst)
            A, b = O.posterior_system(p)
            mu = O.direct_solve(A, b)
            vals.append(float(np.sqrt(np.mean((mu - p.truth.ravel()) ** 2))))
            print(n, inst, vals[-1], flush=True)
        out["rmse_exact"][str(n)] = vals
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table2_exact_rmse.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
