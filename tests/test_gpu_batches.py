"""GPU parity of the recompression when its workspace holds only a small part
of the interpolated couplings: block weights, both total-weight passes,
truncation and projection then run in many workspace batches, and the stacked
rows of a (cluster, direction) pair are folded over several batches (the path
every large problem takes; Section 3.2, total weights of eq.
(recomp_weight_full)).  The results must match the FP64 oracle exactly as the
single-batch builds do: singular values to 1e-12, ranks up to near-ties,
R^* R and Zhat^* Zhat to 1e-12 / 1e-11, matvec to 1e-10."""
import numpy as np
import pytest

import synth
from tests.gpu_common import (say, oracle_for, build_handle, rel, check_ranks_and_sigma,
                               check_weight_invariants)

pytestmark = pytest.mark.gpu

# workspace in GB: a few dozen interpolated couplings per batch
TINY = {"dir2k": 0.002, "cube1200dir": 0.002, "sphere2k": 0.01}


@pytest.mark.parametrize("name", list(TINY))
def test_recompression_in_many_batches_matches_oracle(name):
    import torch
    o = oracle_for(name)
    h, slots = build_handle(name, workspace_gb=TINY[name])
    try:
        s = h.stats()
        say("[gpu] %s workspace %.3f GB: batches basis %d block %d total row %d col %d trunc %d proj %d, "
            "straddled slots %d, S_b regeneration %.2f"
            % (name, TINY[name], s["batches_basis_weights"], s["batches_block_weights"],
               s["batches_total_weights_row"], s["batches_total_weights_col"], s["batches_truncation"],
               s["batches_projection"], s["slots_straddled"], s["coupling_regeneration"]))
        assert s["batches_block_weights"] > 1
        assert s["batches_total_weights_row"] > 1 and s["batches_total_weights_col"] > 1
        assert s["batches_projection"] > 1
        assert s["slots_straddled"] > 0
        check_ranks_and_sigma(h, slots, o, name + " small workspace")
        check_weight_invariants(h, slots, o, name + " small workspace")
        X = synth.complex_gaussian(o.n, 3, seed=0)
        Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        err = rel(Yd.cpu().numpy(), o.matvec(X.T).T)
        say("[gpu] %s small workspace matvec rel err %.3e" % (name, err))
        assert err <= 1e-10
    finally:
        h.free()
