"""DBHT clustering (host, tmfg_dbht) of TMFGs built on the GPU, against the oracle on the same
W bytes and record, for the 200- and 5000-vertex planted-cluster workloads."""
import numpy as np
import pytest
import torch

import oracle
from oracle import dbht as dh
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,flags", [("config_c1", 0), ("config_c2", 0), ("config_c2", "paper")])
def test_dbht_of_gpu_builds(cfg, flags):
    s = getattr(synth, cfg)()
    fl = tm.RULE_PAPER if flags == "paper" else 0
    res = tm.build(X=to_dev(s.X), keep_w=True, flags=fl)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0
    k = len(set(s.labels.tolist()))
    lib = tm.dbht(got["W"], got["order"], got["edges"], got["steps"], k)
    ref = dh.dbht(got["W"], got, k)
    for key in ("labels", "group", "bubble", "linkage"):
        assert np.array_equal(np.asarray(lib[key]), np.asarray(ref[key])), key
    score = dh.ari(s.labels, lib["labels"])
    print(f"{cfg} {flags or 'exact'}: ARI {score:.4f}, converging bubbles {len(set(lib['group'].tolist()))}",
          flush=True)
    assert score > 0.5
