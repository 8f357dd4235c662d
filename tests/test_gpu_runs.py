"""R independent runs at once (ns_run_many): each context on its own stream
and host thread gives exactly the run it gives alone (same seed, same draws,
same decisions), for the fused slice kernel and for the batched rounds."""
import numpy as np
import pytest
import torch

from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("R", [2, 8])
def test_concurrent_rosenbrock_runs_equal_single_runs(R):
    spec = W.likelihood(2)
    kw = dict(prec="f64", state="f32", tree_depth=2)
    streams = [torch.cuda.Stream() for _ in range(R)]
    many = [native.Sampler(spec, 500, seed=10 + r, stream=streams[r], **kw) for r in range(R)]
    rc, steps = native.run_many(many, 50)
    assert rc == native.NS_DONE and np.all(steps > 300)
    for r in range(R):
        one = native.Sampler(spec, 500, seed=10 + r, **kw)
        one.run(50)
        a, b = many[r].dead(), one.dead()
        assert np.array_equal(a["logL"], b["logL"]) and np.array_equal(a["u"], b["u"])
        assert many[r].logZ() == one.logZ()
        assert many[r].stats()["evals"] == one.stats()["evals"]
        one.close()
    for s in many:
        s.close()


def test_concurrent_rounds_runs_equal_single_runs():
    spec = W.likelihood(3, seed=0)
    kw = dict(prec="f32", state="f32", tree_depth=3, batch_rounds=1)
    streams = [torch.cuda.Stream() for _ in range(4)]
    many = [native.Sampler(spec, 1000, seed=r, stream=streams[r], **kw) for r in range(4)]
    native.run_many(many, 100, max_steps=40)
    for r in range(4):
        one = native.Sampler(spec, 1000, seed=r, **kw)
        one.run(100, max_steps=40)
        assert np.array_equal(many[r].dead()["logL"], one.dead()["logL"])
        one.close()


def test_run_many_rejects_a_repeated_context():
    s = native.Sampler(W.likelihood(1), 100, seed=0)
    with pytest.raises(native.NsError, match="NS_EINVAL"):
        native.run_many([s, s], 1)
