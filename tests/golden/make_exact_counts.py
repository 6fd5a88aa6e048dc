"""Write tests/golden/exact_counts.json: exact eigenvalue counts of the
synthetic workloads, computed only with oracle.exact (dense symmetric
eigendecomposition for small n; for larger 3D grids the multifrontal
nested-dissection LDL^T, Sylvester inertia).

Usage: python tests/golden/make_exact_counts.py [names...]
  names: workload names (c1, c2_small, c2_ragged, c2, c3, c5) or "c4" for
  the 64 problems of the batched family (4 shifts each).
(64^3 takes about 2 minutes on 8 cores, 96^3 about 10, 128^3 about an hour.)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from paper_1602_02306_amd import workloads as W  # noqa: E402  (input builder only)

OUT = os.path.join(HERE, "exact_counts.json")


def negcounts(dims, V, A, taus):
    n = int(A.n)
    if n <= 4096:
        Ad = A.to_dense()
        return [exact.dense_negcount(Ad, t) for t in taus], "dense eigvalsh"
    if len(dims) == 3:
        return ([exact.nd_negcount(dims, V, t) for t in taus],
                "nested-dissection LDL^T inertia (Bunch-Kaufman fronts)")
    As = A.to_scipy()
    return [exact.sparse_negcount(As, t) for t in taus], "sparse LDL^T inertia (SuperLU, diagonal pivots)"


def save(data):
    tmp = OUT + ".tmp"
    json.dump(data, open(tmp, "w"), indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        if name == "c4":
            items = data.get("c4", {}).get("items", [])
            for b in range(len(items), 64):
                it = W.batched_item(b)
                neg, method = negcounts(it.dims, it.V, it.A, [float(t) for t in it.shifts])
                items.append({"problem": b, "dims": list(it.dims), "shifts": [float(t) for t in it.shifts],
                              "negcounts": neg, "counts": [neg[i + 1] - neg[i] for i in range(3)],
                              "method": method})
                data["c4"] = {"items": items, "base_seed": 1000}
                save(data)
                print("c4 problem", b, it.dims, neg, "%.0f s" % (time.time() - t0), flush=True)
            continue
        wl = W.WORKLOADS[name]
        P = W.make_problem(wl)
        (a, b), method = negcounts(wl.dims, P.V, P.A, [wl.xi, wl.eta])
        data[name] = {"xi": wl.xi, "eta": wl.eta, "negcount_xi": a, "negcount_eta": b,
                      "count": b - a, "method": method, "dims": list(wl.dims),
                      "potential_seed": wl.seed}
        print(name, data[name], "%.0f s" % (time.time() - t0), flush=True)
        save(data)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2_small", "c2_ragged", "c2"])
