"""Streams and threads: each context enqueues all its work on its own stream,
and contexts are independent.

Two host threads each own a context on its own (default-priority) stream and
solve repeatedly at the same time; every solve must give the levels and the
iterate of the same solve run alone on the default stream, bit for bit.  A
third case hands the solver an iterate produced on another stream: the
binding orders the library's stream after it.
"""
import threading

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problems():
    rng = np.random.default_rng(11)
    return [workloads.poisson([300, 200], b=rng.uniform(-1, 1, (1, 200, 300))),
            workloads.variable_coefficient(24, seed=3, corr_len=3.0)]


def _alone(prob, **kw):
    from paper_2011_06636_amd.solver import Solver
    s = Solver(prob)
    out = s.solve(**kw)
    res = (out["levels"].copy(), out["x"].cpu().numpy())
    s.close()
    return res


def test_two_contexts_two_streams_two_threads(torch_cuda):
    from paper_2011_06636_amd.solver import Solver
    torch = torch_cuda
    probs = _problems()
    kw = dict(tol=1e-9, max_cycles=400)
    ref = [_alone(p, **kw) for p in probs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got, errors = [[], []], []

    def run(k):
        try:
            with torch.cuda.stream(streams[k]):
                s = Solver(probs[k], stream=streams[k])
                for _ in range(3):
                    x = s.zeros()
                    out = s.solve(x, **kw)
                    got[k].append((out["levels"].copy(), x.cpu().numpy()))
                s.close()
        except Exception as e:  # reported below, in the main thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for k in range(2):
        assert len(got[k]) == 3
        for levels, x in got[k]:
            assert np.array_equal(levels, ref[k][0])
            assert np.array_equal(x, ref[k][1])


def test_iterate_from_another_stream(torch_cuda):
    from paper_2011_06636_amd.solver import Solver
    torch = torch_cuda
    prob = _problems()[0]
    kw = dict(tol=1e-9, max_cycles=400)
    ref = _alone(prob, **kw)
    side = torch.cuda.Stream()
    s = Solver(prob, stream=torch.cuda.Stream())
    with torch.cuda.stream(side):
        # a large fill queued ahead on the caller's stream, then the zero start
        pad = torch.empty(1 << 26, dtype=torch.float64, device="cuda").fill_(1.0)
        x = torch.full(prob.shape, 7.0, dtype=torch.float64, device="cuda")
        x.zero_()
        out = s.solve(x, **kw)
        got = x.cpu().numpy()
    s.close()
    del pad
    assert np.array_equal(out["levels"], ref[0])
    assert np.array_equal(got, ref[1])
