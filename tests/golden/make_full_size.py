"""Writes full_size.json: the oracle's result digests for the full-size
single-image workloads (lambda-leveling, and the lambda-skeleton of the ridge
image), so GPU tests can check bit-exactness at sizes where
the oracle takes about a minute.

For each workload it stores the SHA-256 of the generated input (so a test
can tell whether the generator reproduced the same image on its machine),
the SHA-256 of ORACLE-SWEEP-DIRTY's output, and its pass and lowering
counts.  Only the input generators and the oracle are called.

    python tests/golden/make_full_size.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1603_09180_amd import synth  # noqa: E402

WORKLOADS = {
    "ridges_512": synth.ridges_512,
    "blobs_8192_u16": synth.blobs_8192_u16,
    "skeleton_512": synth.skeleton_512,
}


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    oracle.build(force=False)
    out = {}
    for name, make in WORKLOADS.items():
        job = make()
        F = job.image()
        ref = oracle.sweep_dirty(F, job.lam, job.adj, op=job.op)
        out[name] = {"h": int(F.shape[0]), "w": int(F.shape[1]), "dtype": str(F.dtype),
                     "lambda": int(job.lam), "adjacency": int(job.adj), "op": job.op,
                     "input_sha256": digest(F), "output_sha256": digest(ref.image),
                     "passes": int(ref.passes), "lowerings": int(ref.lowerings)}
        print(name, out[name], flush=True)
    with open(os.path.join(HERE, "full_size.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
