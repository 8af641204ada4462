"""Write the oracle's direct FP64 end-point forces on sampled segments of the
large loop ensembles to tests/golden/oracle_samples_<workload>.json.

Only the oracle and the seeded generator are called.  The GPU tests compare
the FMM forces at full size with these values (global relative L2 error over
the sample).  Usage: python tests/golden/make_golden.py [workload ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLES = {"iso200k": 60, "cubic100k": 16, "cubic1m": 64}
SEED = 424242


def main(names):
    for name in names:
        seg, b, prm = synth.make_workload(name)
        tgt = synth.segment_subset(seg.shape[0], SAMPLES[name], SEED)
        t0 = time.time()
        f = oracle.direct_forces(seg, b, oracle.medium_from_params(prm), targets=tgt)
        out = {"workload": name, "n_seg": int(seg.shape[0]), "subset_seed": SEED, "n_quad": 3,
               "n_circle": 64, "targets": [int(x) for x in tgt],
               "forces": [[[float(v) for v in end] for end in fs] for fs in f],
               "oracle_seconds": time.time() - t0, "oracle_threads": oracle.num_threads()}
        path = os.path.join(ROOT, "tests", "golden", "oracle_samples_%s.json" % name)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=0)
        print(name, "%.1f s" % out["oracle_seconds"], path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(SAMPLES))
