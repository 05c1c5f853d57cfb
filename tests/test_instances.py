"""The torch and NumPy forms of the seeded generator draw identical values."""
import numpy as np
import pytest
import torch

from paper_2305_07187_amd import instances


def test_splitmix_streams_agree():
    for seed in (0, 1, 12345, 2 ** 63 + 7):
        a = instances.splitmix64(seed, 1000)
        b = instances.splitmix64_torch(seed, 1000, "cpu").numpy().view(np.uint64)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [2, 17, 130])
def test_instances_agree(n):
    for kind in ("pm1", "gauss"):
        a = instances.make_J(n, kind, 5)
        b = instances.make_J_torch(n, kind, 5, "cpu").numpy()
        assert np.array_equal(a, b), kind
    assert np.array_equal(instances.make_x0(n, 7, 3), instances.make_x0_torch(n, 7, 3, device="cpu").numpy())


def test_batch_recipe_range():
    b = instances.make_batch(256, 0)
    ns = [x[0] for x in b]
    assert min(ns) >= 64 and max(ns) <= 4096 and len(set(ns)) > 100
    assert [x[1] for x in b[:4]] == ["pm1", "gauss", "pm1", "gauss"]
