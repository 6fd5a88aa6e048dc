"""Write tests/golden/exact_counts.json: exact eigenvalue counts of the
synthetic workloads, computed only with oracle.exact (dense symmetric
eigendecomposition for small n, sparse LDL^T Sylvester inertia otherwise).

Usage: python tests/golden/make_exact_counts.py [names...]
(the 64^3 case takes about 10 minutes on 8 cores).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from paper_1602_02306_amd import workloads as W  # noqa: E402  (input builder only)

OUT = os.path.join(HERE, "exact_counts.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        wl = W.WORKLOADS[name]
        P = W.make_problem(wl)
        if wl.n <= 4096:
            Ad = P.A.to_dense()
            a, b = exact.dense_negcount(Ad, wl.xi), exact.dense_negcount(Ad, wl.eta)
            method = "dense eigvalsh"
        else:
            As = P.A.to_scipy()
            a, b = exact.sparse_negcount(As, wl.xi), exact.sparse_negcount(As, wl.eta)
            method = "sparse LDL^T inertia (SuperLU, diagonal pivots)"
        data[name] = {"xi": wl.xi, "eta": wl.eta, "negcount_xi": a, "negcount_eta": b,
                      "count": b - a, "method": method, "dims": list(wl.dims),
                      "potential_seed": wl.seed}
        print(name, data[name], flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2_small", "c2_ragged", "c2"])
