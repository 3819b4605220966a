"""Helpers shared by the GPU tests: run the HIP evaluator and the oracle on
the same seeded net and compare element by element."""
import numpy as np

import oracle
import paper_1404_0076_amd as P


def oracle_run(rules, net):
    return oracle.reduce(rules, net)


def assert_same(gpu, ref, what=""):
    res, nf, pr = gpu
    assert res.status == ref.status, f"{what}: status {res.status} vs {ref.status}"
    assert res.interactions == ref.interactions, f"{what}: {res.interactions} vs {ref.interactions}"
    assert np.array_equal(pr.astype(np.uint64), ref.per_rule.astype(np.uint64)), f"{what}: per-rule"
    assert res.n_stuck == ref.n_stuck, what
    assert len(nf) == len(ref.nf), f"{what}: stream length {len(nf)} vs {len(ref.nf)}"
    assert np.array_equal(nf, ref.nf), f"{what}: first difference at {np.argmax(nf != ref.nf)}"
