"""The learned encoder and the radiance evaluation captured in a HIP graph:
every replay (with eager work of the program between replays) reproduces the
eager result bit for bit.  The encoder's only buffer resets are kernels, so
the captured graph holds kernel nodes only."""
import numpy as np
import pytest
import torch

from paper_2605_30396_amd import inputs as I
from paper_2605_30396_amd import sc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_learned_encode_and_radiance_replay_in_a_graph():
    rng = I.rng_for(700)
    N, K, k, eps = 50_000, 256, 12, 1e-2
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, N, 4, 1e-3)
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    p = sc.proposer_create(45, 256, K)
    p.set_params(I.mlp_init(I.rng_for(701), 45, 256, K))
    Xg = torch.from_numpy(X).to(DEV)
    dirs = torch.from_numpy(I.unit_directions(I.rng_for(702), N)).to(DEV)
    out = (torch.empty((N, k), dtype=torch.int32, device=DEV), torch.empty((N, k), dtype=torch.float32, device=DEV),
           torch.empty((N,), dtype=torch.int32, device=DEV), torch.empty((N,), dtype=torch.float32, device=DEV))
    ws = torch.empty(sc.learned_workspace_bytes(N, 24), dtype=torch.uint8, device=DEV)
    rgb = torch.empty((N, 3), dtype=torch.float32, device=DEV)

    def step():
        sc.omp_encode_learned(h, p, Xg, k, eps, out=out, workspace=ws)
        sc.sh_eval_sparse(h, out[0], out[1], out[2], dirs, sc.DIRS_PER_SIGNAL, out=rgb)

    step()   # eager: also performs the one-time launch set-up outside the capture
    torch.cuda.synchronize()
    ref = [t.clone() for t in out] + [rgb.clone()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        for t in list(out) + [rgb]:
            t.fill_(7)   # eager work between replays, clobbering the outputs
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(list(out) + [rgb], ref):
            assert torch.equal(a, b), f"replay {rep} differs from the eager result"
    p.destroy()
    h.destroy()
