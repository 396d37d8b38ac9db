"""Host logic of the surrogate pipeline that needs no GPU: the ordering key
of the labelling walks (the length of an item's longest walks)."""
import numpy as np

from paper_2409_00165_amd import surrogate_pipeline as SP
from paper_2409_00165_amd import workloads as W


def _items(tau_s, tau_a, g, t=100.0):
    n = len(tau_s)
    return {"thickness": np.full((n, 1), t), "mu_s": (np.asarray(tau_s, float) / t)[:, None],
            "mu_a": (np.asarray(tau_a, float) / t)[:, None], "g": np.asarray(g, float)[:, None]}


def test_walk_cost_is_diffusion_time_or_scatterings_before_absorption():
    # thick and lossless: tau_s^2 (1 - g) scatterings, i.e. (tau_s (1 - g))^2
    # transport paths of 1 / (1 - g) scatterings; strongly absorbing:
    # tau_s / tau_a; thin: at least 1
    c = SP._walk_cost(_items([1e4, 1e4, 1e4, 0.1], [1e-4, 10.0, 1e-4, 1e-4], [0.0, 0.0, 0.9, 0.0]))
    assert np.allclose(c, [1e8, 1e3, 1e7, 1.0])


def test_label_launch_sizes_cover_the_items_longest_first():
    sizes = SP.label_launch_sizes(2_000_000)
    assert sum(sizes) == 2_000_000 and sizes[:4] == [1024, 1024, 2048, 2048]
    assert max(sizes) == 262_144 and all(s > 0 for s in sizes)
    assert SP.label_launch_sizes(3000) == [1024, 1024, 952]
    assert sum(SP.label_launch_sizes(20_000)) == 20_000


def test_walk_cost_orders_the_training_recipe_longest_first():
    a = W.surrogate_training_items(20000, 5)
    c = SP._walk_cost(a)
    order = np.argsort(-c, kind="stable")
    t = a["thickness"][:, 0]
    tau_red = a["mu_s"][:, 0] * t * (1 - a["g"][:, 0])
    # the first percent of the order holds the thickest reduced depths of the recipe
    head = order[: len(order) // 100]
    assert np.median(tau_red[head]) > np.quantile(tau_red, 0.9)
    assert np.all(np.isfinite(c)) and np.all(c >= 0)


def test_label_streams_give_the_first_launch_a_stream_of_its_own():
    from paper_2409_00165_amd import surrogate_pipeline as SP
    assert [SP.label_stream(j, 1) for j in range(5)] == [0, 0, 0, 0, 0]
    assert [SP.label_stream(j, 2) for j in range(5)] == [0, 1, 1, 1, 1]
    got = [SP.label_stream(j, 8) for j in range(22)]
    assert got[0] == 0 and 0 not in got[1:]
    assert got[1:8] == [1, 2, 3, 4, 5, 6, 7] and got[8:15] == [1, 2, 3, 4, 5, 6, 7]
