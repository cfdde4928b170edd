"""Writes batch_512.json: the oracle's per-image result digests for the
512-image batch workload (uneven u8 blob images, sides log-uniform in
64..2048, lambda from {0, 5, 20, 50}, (8,4), image seeds 4000 + i), so the
GPU test and the benchmark can check every image of the batch bit for bit.

For each image it stores the generator parameters, the SHA-256 of the
generated input (a consumer can tell whether the generator reproduced the
same image on its machine), the SHA-256 of ORACLE-SWEEP-DIRTY's output, its
pass, lowering and examination counts.  Only the input generators and the
oracle are called; the images are independent, so they are spread over a
process pool.

    python tests/golden/make_batch_512.py [workers]
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def one(i: int):
    import oracle
    from paper_1603_09180_amd import synth

    job = synth.batch_512_uneven()[i]
    F = job.image()
    t0 = time.perf_counter()
    ref = oracle.sweep_dirty(F, job.lam, job.adj)
    dt = time.perf_counter() - t0
    return {"i": i, "h": job.h, "w": job.w, "lambda": job.lam, "adjacency": job.adj,
            "seed": job.seed, "input_sha256": digest(F), "output_sha256": digest(ref.image),
            "passes": int(ref.passes), "lowerings": int(ref.lowerings),
            "examinations": int(ref.examinations), "oracle_s": round(dt, 3)}


def main():
    import oracle
    from paper_1603_09180_amd import synth

    oracle.build(force=False)
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    n = len(synth.batch_512_uneven())
    # largest images first, so the pool drains evenly
    jobs = synth.batch_512_uneven()
    order = sorted(range(n), key=lambda i: -jobs[i].h * jobs[i].w)
    t0 = time.perf_counter()
    with mp.Pool(workers) as pool:
        recs = []
        for k, rec in enumerate(pool.imap_unordered(one, order)):
            recs.append(rec)
            if k % 64 == 63:
                print(f"{k + 1}/{n} images, {time.perf_counter() - t0:.0f} s", flush=True)
    recs.sort(key=lambda r: r["i"])
    out = {"workload": "batch_512", "generator": "synth.batch_512_uneven()", "images": recs,
           "total_pixels": int(sum(r["h"] * r["w"] for r in recs)),
           "oracle_cpu_s": round(sum(r["oracle_s"] for r in recs), 1)}
    with open(os.path.join(HERE, "batch_512.json"), "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"wrote {len(recs)} records in {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
