"""Writes sh_like_dict_K256.npy: the K=256 dictionary of the SH-like workload.

It is learned by the FP64 oracle's alternating minimisation (OMP codes, then
the least-squares dictionary update, 10 passes; Sec. 2.1) on the first 100,000
SH-like signals (seed 2), with k=8 and eps=1e-3.  Run from the repository
root:  python tests/golden/make_sh_like_dictionary.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2605_30396_amd import inputs as I  # noqa: E402


def main():
    X = I.sh_like_signals(I.rng_for(2), 1_000_000)[:100_000]
    D, hist = oracle.mod_learn(X, K=256, k=8, eps=1e-3, passes=10, seed=2)
    path = os.path.join(HERE, "sh_like_dict_K256.npy")
    np.save(path, D)
    meta = dict(file="sh_like_dict_K256.npy", shape=list(D.shape), dtype="float32",
                sha256=hashlib.sha256(D.tobytes()).hexdigest(),
                recipe="oracle.mod_learn(first 100k of sh_like_signals(seed 2), K=256, k=8, eps=1e-3, passes=10, seed=2)",
                mean_sq_residual_per_pass=hist)
    with open(os.path.join(HERE, "sh_like_dict_K256.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta, indent=1))


if __name__ == "__main__":
    main()
