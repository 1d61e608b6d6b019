"""Host logic of the batch split into plans by spatial order (no GPU):
split_by_order partitions the pairs (each exactly once, listed orders first,
empty groups dropped) and the tuner's candidates are the documented splits."""
from paper_1901_09999_amd import psfm, tune


def _pairs(orders):
    return [dict(S=s) for s in orders]


def test_split_by_order_partitions_the_pairs():
    pairs = _pairs([0, 3, 2, 1, 3, 0, 2, 3])
    plans = psfm.split_by_order(pairs, [[3], [2]])
    assert plans == [[1, 4, 7], [2, 6], [0, 3, 5]]
    assert sorted(k for ix in plans for k in ix) == list(range(len(pairs)))
    # no groups: one plan of everything
    assert psfm.split_by_order(pairs, []) == [list(range(len(pairs)))]
    # a listed order with no pairs and an empty remainder are dropped
    assert psfm.split_by_order(_pairs([1, 1, 2]), [[3], [2], [1]]) == [[2], [0, 1]]
    # orders may share a group
    assert psfm.split_by_order(pairs, [[3, 2]]) == [[1, 2, 4, 6, 7], [0, 3, 5]]


def test_order_group_candidates():
    assert tune.order_groups(_pairs([0, 0])) == [[]]
    assert tune.order_groups(_pairs([0, 2])) == [[], [[2]]]
    assert tune.order_groups(_pairs([1, 0, 2])) == [[], [[2]], [[2], [1]]]
    assert tune.order_groups(_pairs([0, 1, 2, 3, 3])) == [[], [[3]], [[3], [2]], [[3], [2], [1]]]
    # every candidate splits the pairs into a partition
    pairs = _pairs([3, 0, 1, 2, 2, 3])
    for g in tune.order_groups(pairs):
        plans = psfm.split_by_order(pairs, g)
        assert sorted(k for ix in plans for k in ix) == list(range(len(pairs)))
