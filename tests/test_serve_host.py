"""Host logic of the serving runtime: HBM admission and the batch selection policy."""
import collections

import pytest

from paper_1605_02406_amd.serve import Admission, Request, select_batch


def test_admission_budget():
    a = Admission(1000)
    assert a.try_reserve("a", 600)
    assert not a.try_reserve("b", 401)   # one byte over what is left
    assert a.try_reserve("b", 400)       # exact fit
    assert a.free == 0 and a.used == 1000
    assert not a.try_reserve("c", 1)
    assert a.release("a") == 600
    assert a.try_reserve("c", 600)
    with pytest.raises(KeyError):
        a.try_reserve("c", 1)            # one reservation per stream
    with pytest.raises(KeyError):
        a.release("zz")
    with pytest.raises(ValueError):
        Admission(-1)


def test_zero_budget_admits_only_empty_reservations():
    a = Admission(0)
    assert not a.try_reserve("a", 1)
    assert a.try_reserve("b", 0)


def _pending(spec):
    """spec: {sid: [arrival times]} -> pending queues in insertion order."""
    p = collections.OrderedDict()
    for sid, times in spec.items():
        p[sid] = collections.deque(Request(sid, None, t, i) for i, t in enumerate(times))
    return p


def test_batch_takes_the_oldest_head_of_each_stream():
    p = _pending({"a": [3.0, 4.0], "b": [1.0, 1.5, 9.0], "c": [2.0], "d": []})
    assert select_batch(p, 32) == ["b", "c", "a"]   # each stream once, by head arrival
    assert select_batch(p, 2) == ["b", "c"]
    assert select_batch(p, 1) == ["b"]
    assert select_batch(collections.OrderedDict(), 4) == []


def test_batch_ties_keep_insertion_order():
    p = _pending({"x": [1.0], "y": [1.0], "z": [0.5]})
    assert select_batch(p, 3) == ["z", "x", "y"]

