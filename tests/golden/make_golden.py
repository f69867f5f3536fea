"""Write oracle log-likelihoods for sampled templates of the full-size workloads.

Calls only ``synth`` (inputs) and ``oracle`` (FP64 reference).  Run from the repo
root:  python tests/golden/make_golden.py
Outputs tests/golden/{c2,c3,c2_stress}_sample.json: the sampled template rows, the
oracle's network logL for them, log det and N_eff per detector, and the input recipe
(c2_stress: the two-detector N = 16384 workload at the stress nugget 1e-8), and
tests/golden/c4_sample.json: the same for sampled rows of sampled instances of the
64-instance ragged workload.
"""
import json
import os
import sys
import time

# The threaded OpenBLAS shipped with numpy/scipy here segfaults in the Cholesky of the
# ~32k x 32k gapped block; single-threaded BLAS factors it correctly (slower).
if "c3" in sys.argv[1:] or "c4" in sys.argv[1:] or len(sys.argv) == 1:
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLE = {"c2": [0, 1, 2, 511, 1024, 2047, 2048, 3071, 4000, 4095],
          "c3": [0, 1, 100, 2047, 4096, 5000, 8000, 8191]}
SAMPLE["c2_stress"] = SAMPLE["c2"]
# C4: instances of N <= 14000 (one or two detectors, with and without gaps), three rows each
C4_INSTANCES = [0, 2, 3, 15, 24]
C4_ROWS = [0, 100, 255]


def run_c4():
    t = time.time()
    w = synth.c4_workload()
    out = {"workload": "c4", "instances": C4_INSTANCES, "rows": C4_ROWS, "items": [],
           "eps": w.instances[0].eps,
           "recipe": "synth.c4_workload(); per sampled instance oracle.factor per detector + "
                     "oracle.loglik_network on the sampled rows"}
    for i in C4_INSTANCES:
        inst = w.instances[i]
        fs = [oracle.factor(inst.acf, inst.N, inst.masks[k]) for k in range(inst.n_det)]
        ll = oracle.loglik_network(fs, inst.d, inst.H[C4_ROWS])
        out["items"].append({"instance": i, "N": inst.N, "n_det": inst.n_det,
                             "loglik": [float(x) for x in ll],
                             "logdet": [f.logdet for f in fs], "n_eff": [f.n_eff for f in fs]})
    with open(os.path.join(HERE, "c4_sample.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("c4 done in %.0f s" % (time.time() - t), flush=True)


def run(name):
    if name == "c4":
        return run_c4()
    rows = SAMPLE[name]
    t = time.time()
    if name == "c3":
        w = synth.c3_workload(rows=rows)
    else:
        w = synth.c2_workload(rows=rows, eps=synth.EPS_STRESS if name == "c2_stress"
                              else synth.EPS_PRIMARY)
    inst = w.instances[0]
    fs = [oracle.factor(inst.acf, inst.N, inst.masks[k]) for k in range(inst.n_det)]
    ll = oracle.loglik_network(fs, inst.d, inst.H)
    out = {"workload": name, "N": inst.N, "n_det": inst.n_det, "eps": inst.eps,
           "rows": rows, "loglik": [float(x) for x in ll],
           "logdet": [f.logdet for f in fs], "n_eff": [f.n_eff for f in fs],
           "recipe": "synth.%s_workload(rows=rows%s); oracle.factor + oracle.loglik_network"
                     % (name[:2], ", eps=synth.EPS_STRESS" if name == "c2_stress" else "")}
    with open(os.path.join(HERE, f"{name}_sample.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "done in %.0f s" % (time.time() - t), flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["c2", "c3", "c2_stress", "c4"]):
        run(n)
