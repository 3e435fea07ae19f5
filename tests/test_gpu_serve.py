"""Serving on the GPU: streams of different sizes served in a mix (continuous batching, requests
in arrival order across batches) end in exactly the state each reaches stepped alone; admission
refuses a stream whose arena does not fit the budget."""
import numpy as np
import pytest
import torch

from paper_1605_02406_amd import dogm, scenes
from paper_1605_02406_amd.serve import Server
from tests.parity import device_meas, host

pytestmark = pytest.mark.gpu

SIZES = [(24, 24), (64, 64), (40, 17), (96, 96), (32, 32)]
CYCLES = 4


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dogm.lib()


def _params(i, nx, ny):
    f = dict(scenes.FILTER)
    return dogm.make_params(nx, ny, 0.2, 8 * nx * ny, nx * ny, seed=100 + i, grid_id=i, **f)


def _sequences():
    out = []
    for i, (nx, ny) in enumerate(SIZES):
        wl = dict(nx=nx, ny=ny, cell=0.2, n_pers=8 * nx * ny, n_born=nx * ny, scene="boxes",
                  n_boxes=3, clutter=0.01, seed=i)
        out.append([device_meas(m) for m in scenes.measurement_sequence(wl, CYCLES, seed=i)])
    return out


def _alone(seqs):
    ref = []
    for i, (nx, ny) in enumerate(SIZES):
        g = dogm.Grid(_params(i, nx, ny))
        for m in seqs[i]:
            g.step(m)
        torch.cuda.synchronize()
        ref.append({k: host(v).copy() for k, v in g.v.items()})
    return ref


def test_served_mix_equals_each_stream_alone():
    seqs = _sequences()
    ref = _alone(seqs)
    budget = sum(dogm.arena_bytes(_params(i, nx, ny)) for i, (nx, ny) in enumerate(SIZES))
    srv = Server(budget, max_batch=3, max_inflight=2)
    for i, (nx, ny) in enumerate(SIZES):
        assert srv.open(i, _params(i, nx, ny))
    # arrivals: every stream's cycles in order, streams interleaved at random
    rng = np.random.default_rng(5)
    order = [i for i in range(len(SIZES)) for _ in range(CYCLES)]
    rng.shuffle(order)
    nxt = [0] * len(SIZES)
    for t, i in enumerate(order):
        srv.submit(i, seqs[i][nxt[i]])
        nxt[i] += 1
        if t % 3 == 0:
            srv.pump()
    srv.drain()
    assert len(srv.stats.done) == len(order)
    assert srv.stats.batches >= len(order) // 3
    for i in range(len(SIZES)):
        seqs_done = [r.seq for r in srv.stats.done if r.sid == i]
        assert seqs_done == list(range(CYCLES))
        g = srv.grids[i]
        assert g.cycle == CYCLES + 1
        for k, v in g.v.items():
            assert np.array_equal(host(v), ref[i][k]), (i, k)
    for r in srv.stats.done:
        assert r.t_arrival <= r.t_launch <= r.t_done, (r.sid, r.seq)


def test_admission_refuses_over_budget_and_frees_on_close():
    p_small, p_big = _params(0, 24, 24), _params(1, 96, 96)
    b_small, b_big = dogm.arena_bytes(p_small), dogm.arena_bytes(p_big)
    srv = Server(b_big + b_small - 1)
    assert srv.open("big", p_big)
    assert not srv.open("small", p_small)
    assert srv.stats.rejected_streams == 1 and "small" not in srv.grids
    srv.close("big")
    assert srv.admission.used == 0
    assert srv.open("small", p_small)
    with pytest.raises(KeyError):
        srv.submit("big", None)


def test_close_waits_only_for_the_closed_stream():
    """Closing a stream with a cycle in flight finishes that cycle and keeps the other streams'
    queued requests queued."""
    seqs = _sequences()
    srv = Server(1 << 34, max_batch=1, max_inflight=2)
    for i in (0, 1):
        assert srv.open(i, _params(i, *SIZES[i]))
    srv.submit(0, seqs[0][0])
    srv.pump()                      # stream 0 in flight
    srv.submit(1, seqs[1][0])      # stream 1 queued behind it
    srv.close(0)
    assert 0 not in srv.grids and srv.admission.used == dogm.arena_bytes(_params(1, *SIZES[1]))
    assert [r.sid for r in srv.stats.done] == [0]
    assert list(srv.pending) == [1]
    srv.drain()
    assert [r.sid for r in srv.stats.done] == [0, 1]
    with pytest.raises(KeyError):
        srv.close(0)
