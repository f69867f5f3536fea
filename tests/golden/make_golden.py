"""Write oracle log-likelihoods for sampled templates of the full-size workloads.

Calls only ``synth`` (inputs) and ``oracle`` (FP64 reference).  Run from the repo
root:  python tests/golden/make_golden.py
Outputs tests/golden/{c2,c3}_sample.json: the sampled template rows, the oracle's
network logL for them, log det and N_eff per detector, and the input recipe.
"""
import json
import os
import sys
import time

# The threaded OpenBLAS shipped with numpy/scipy here segfaults in the Cholesky of the
# ~32k x 32k gapped block; single-threaded BLAS factors it correctly (slower).
if "c3" in sys.argv[1:] or len(sys.argv) == 1:
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLE = {"c2": [0, 1, 2, 511, 1024, 2047, 2048, 3071, 4000, 4095],
          "c3": [0, 1, 100, 2047, 4096, 5000, 8000, 8191]}


def run(name):
    rows = SAMPLE[name]
    t = time.time()
    w = synth.c2_workload(rows=rows) if name == "c2" else synth.c3_workload(rows=rows)
    inst = w.instances[0]
    fs = [oracle.factor(inst.acf, inst.N, inst.masks[k]) for k in range(inst.n_det)]
    ll = oracle.loglik_network(fs, inst.d, inst.H)
    out = {"workload": name, "N": inst.N, "n_det": inst.n_det, "eps": inst.eps,
           "rows": rows, "loglik": [float(x) for x in ll],
           "logdet": [f.logdet for f in fs], "n_eff": [f.n_eff for f in fs],
           "recipe": "synth.%s_workload(rows=rows); oracle.factor + oracle.loglik_network" % name}
    with open(os.path.join(HERE, f"{name}_sample.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "done in %.0f s" % (time.time() - t), flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["c2", "c3"]):
        run(n)
