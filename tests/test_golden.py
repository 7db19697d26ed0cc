"""Stored expected values (tests/golden/oracle_small.json, written by make_golden.py from the
oracle only): the oracle must keep reproducing them, and the GPU path must match them."""
import json
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
G = json.load(open(os.path.join(HERE, "golden", "oracle_small.json")))


def stored(entry, key):
    return np.asarray(G[entry][key + "_re"]) + 1j * np.asarray(G[entry][key + "_im"])


def test_oracle_reproduces_golden(oracle_mod):
    e = G["cn_plain_1d_24"]
    w = workloads.plain_1d(n=e["n"], dx=e["dx"], dt=e["dt"], steps=e["steps"])
    out = oracle_mod.cn_propagate(w["psi0"], w["V"], w["dx"], w["dt"], w["steps"])
    np.testing.assert_allclose(out, stored("cn_plain_1d_24", "psi"), rtol=0, atol=1e-15)
    a, b, c, d = workloads.random_system(17, G["solve_dd_17"]["seed"], "dd")
    np.testing.assert_allclose(oracle_mod.thomas(a, b, c, d), stored("solve_dd_17", "x"),
                               rtol=0, atol=1e-15)


@pytest.mark.gpu
def test_gpu_matches_golden():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00856_amd as cn

    e = G["cn_plain_1d_24"]
    w = workloads.plain_1d(n=e["n"], dx=e["dx"], dt=e["dt"], steps=e["steps"])
    psi = torch.tensor(w["psi0"], device="cuda")
    V = torch.tensor(w["V"], device="cuda")
    cn.propagate(psi, V, w["dx"], w["dt"], w["steps"])
    ref = stored("cn_plain_1d_24", "psi")
    assert np.linalg.norm(psi.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-11
    a, b, c, d = workloads.random_system(17, G["solve_dd_17"]["seed"], "dd")
    x = cn.solve(*(torch.tensor(v, device="cuda") for v in (a, b, c, d)))
    ref = stored("solve_dd_17", "x")
    assert np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-11
