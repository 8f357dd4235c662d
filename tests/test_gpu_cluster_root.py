"""Trees whose root holds more points than one workgroup keeps in LDS (FP32
state, N d 4 bytes beyond 80 KiB, a split below the root): the root's mean,
covariance and 2-means split come from the multi-workgroup passes, the
deeper nodes from the per-node kernel.  The whole tree equals the oracle's
tree of the same FP32 points (Sec. 2.1): counts, split decisions, accepted
nodes and labels exactly, centres and factors to rounding."""
import numpy as np
import pytest

import oracle
from paper_2608_28514_amd import native, workloads as W

pytestmark = pytest.mark.gpu


def _same_tree(s, lv, depth):
    t_ref, lab_ref = oracle.cluster(lv["u"], depth, nmin=2 * (s.d + 1))
    t = s.tree()
    assert np.array_equal(t["count"], t_ref["count"])
    assert np.array_equal(t["split_ok"], t_ref["split_ok"])
    assert np.array_equal(t["accepted"], t_ref["accepted"])
    ok = t["count"] >= 2
    assert np.allclose(t["centre"][ok], t_ref["centre"][ok], rtol=1e-12, atol=1e-14)
    assert np.allclose(t["chol"][ok], t_ref["chol"][ok], rtol=1e-9, atol=1e-12)
    return t, lab_ref


@pytest.mark.parametrize("depth", [1, 2])
def test_emulator_live_set_tree_equals_oracle(depth):
    """27-d live set of 4000 points (432 KB of FP32 state)."""
    spec = W.likelihood(5, seed=0)
    print(f"cluster root: emulator N=4000 depth={depth}", flush=True)
    s = native.Sampler(spec, 4000, prec="bf16x3", state="f32", tree_depth=depth, seed=4)
    lv = s.live()
    assert np.array_equal(lv["u"], lv["u"].astype(np.float32).astype(np.float64))
    t, lab_ref = _same_tree(s, lv, depth)
    assert np.array_equal(lv["label"], lab_ref)
    assert t["count"][0] == 4000 and t["count"][1] + t["count"][2] == 4000
    s.close()


def test_two_gaussians_trees_along_a_run_equal_oracle():
    """Eq. (3) in 10-d with 3000 live points (120 KB): trees rebuilt along a
    run until the two modes sit in separate accepted nodes."""
    spec = W.paper_problem("test2_two_gauss")
    s = native.Sampler(spec, 3000, prec="f64", state="f32", tree_depth=2, seed=3)
    s.run(300, max_steps=40)
    compared = splits = 0
    for _ in range(200):
        if splits >= 2:
            break
        lv = s.live()
        n_cl = s.stats()["clusterings"]
        s.step(300)
        if s.stats()["clusterings"] == n_cl:
            continue
        print(f"cluster root: two gaussians, tree {compared}", flush=True)
        t, lab_ref = _same_tree(s, lv, 2)
        after = s.live()
        same = np.all(after["u"] == lv["u"], axis=1)
        assert np.array_equal(after["label"][same], lab_ref[same])
        compared += 1
        splits += int(t["accepted"].sum() > 1)
    print(f"two-gaussian trees compared: {compared}, with more than one cluster: {splits}")
    assert splits >= 2
    s.close()


def test_grid_barrier_that_gives_up_stops_the_run_cleanly():
    """The one-launch split waits at grid barriers with a bounded number of
    polls (wait_limit).  With a limit of one poll some barrier usually gives
    up: the run must then stop and report NS_EDEVICE, and the device must
    stay usable; if no barrier gave up, the run is the default run."""
    spec = W.likelihood(5, seed=0)
    ref = native.Sampler(spec, 4000, prec="bf16x3", state="f32", tree_depth=1, seed=4)
    ref.run(400, max_steps=2)
    ref_dead = ref.dead()["logL"]
    ref.close()
    faulted = False
    try:
        s = native.Sampler(spec, 4000, prec="bf16x3", state="f32", tree_depth=1, seed=4, wait_limit=1)
        try:
            s.run(400, max_steps=2)
            assert np.array_equal(s.dead()["logL"], ref_dead)
        finally:
            s.close()
    except native.NsError as e:
        assert "grid barrier" in str(e) or "NS_EDEVICE" in str(e)
        faulted = True
    print(f"wait_limit=1: a barrier gave up: {faulted}")
    again = native.Sampler(spec, 4000, prec="bf16x3", state="f32", tree_depth=1, seed=4)
    again.run(400, max_steps=2)
    assert np.array_equal(again.dead()["logL"], ref_dead)
    again.close()
