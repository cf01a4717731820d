"""Stored fixtures: checksums and the properties their recipes guarantee."""
import hashlib
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_sh_like_dictionary_fixture():
    meta = json.load(open(os.path.join(GOLD, "sh_like_dict_K256.json")))
    D = np.load(os.path.join(GOLD, meta["file"]))
    assert D.shape == (256, 45) and D.dtype == np.float32
    assert hashlib.sha256(D.tobytes()).hexdigest() == meta["sha256"]
    # Eq. (1): unit-norm atoms
    np.testing.assert_allclose(np.linalg.norm(D.astype(np.float64), axis=1), 1.0, atol=1e-6)
    # alternating minimisation lowered the fit error pass after pass
    h = meta["mean_sq_residual_per_pass"]
    assert all(b <= a for a, b in zip(h, h[1:]))
