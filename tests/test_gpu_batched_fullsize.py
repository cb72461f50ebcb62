"""Batched scenes at the size of the sensitivity sweep: 256 independent
funnel scenes of 2,000-60,000 clumps (log-uniform; 4.26M clumps, 15.4M
spheres), in the launch configuration the benchmark times (FP32 force
arithmetic, learned detection interval with the package's envelope MLP,
replay of captured graphs, the autotuner's bin size and launch shape).

Scenes extracted from the batch and run alone evolve bit for bit as inside
it (the largest, a middle-sized and the smallest scene), from a state run
0.05 s into the discharge.  The three smallest scenes, extracted, deposited
into their funnels on the CPU and run in the all-FP64 mode, follow the
oracle bit for bit."""
import os

import numpy as np
import pytest

import bench
import oracle
from paper_2307_03445_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    return I.funnel_batch()


@pytest.fixture(scope="module")
def mlp():
    from paper_2307_03445_amd import train
    p = train.load_weights()
    assert p is not None, "the package's envelope-MLP weights are missing"
    return p


def test_extracted_scenes_evolve_as_in_the_batch_at_full_size(batch, mlp):
    from paper_2307_03445_amd import prep
    assert batch.n_scenes == 256 and batch.n_spheres > 15_000_000
    d, info = prep.settle_funnels(batch, seconds=0.05)
    print(f"settled: {info}", flush=True)
    b = bench.make_scene(d, "learned", mlp)
    b.step(5)
    tune = b.autotune(bench.DETECT["k_max"])  # its trials are ordinary steps of the run
    b.set_graph(20)
    steps = b.counts()["steps"] + 120  # across at least one more audit
    b.step(steps - b.counts()["steps"])
    cb = b.counts()
    sb = b.state()
    contacts = b.last_step_contacts()
    b.close()
    print(f"batch: {cb}, tuned {tune}, {contacts} contact sides on the last step", flush=True)
    assert cb["steps"] == steps and cb["missed"] == 0 and cb["audits"] >= 2
    assert contacts > d.n_clumps // 4  # the clumps have left the spawn lattice and touch
    sizes = np.bincount(d.clump_scene, minlength=d.n_scenes)
    order = np.argsort(sizes, kind="stable")
    for k in (int(order[-1]), int(order[len(order) // 2]), int(order[0])):
        e = I.extract_scene(d, k)
        a = bench.make_scene(e, "learned", mlp)
        a.step(steps)
        ca, sa = a.counts(), a.state()
        a.close()
        sel = np.nonzero(d.clump_scene == k)[0]
        print(f"scene {k}: {len(sel)} clumps, {ca['detections']} detections", flush=True)
        for key in ("x", "q", "v", "w"):
            assert np.array_equal(sa[key], sb[key][sel]), (k, key)
        assert ca["missed"] == 0


def test_smallest_extracted_scenes_match_the_oracle_fp64(batch):
    """The three smallest scenes of the batch, stand-alone, with their clumps
    deposited into their funnels on the CPU (a column on the plate under the
    outlet, the funnel filled above it): first-step contacts, forces and
    histories, then 100-step trajectories, bit-identical to the oracle."""
    from paper_2307_03445_amd._lib import Scene
    from paritylib import compare_pairs
    oracle.set_threads(min(16, os.cpu_count() or 1))
    sizes = np.bincount(batch.clump_scene, minlength=batch.n_scenes)
    for k in np.argsort(sizes, kind="stable")[:3]:
        e = I.funnel_deposited(batch, int(k))
        sc, o = Scene(e, precision="fp64"), oracle.Oracle(e)
        sc.record_next_step()
        sc.step(1)
        o.eval()
        cg, co = sc.contacts(), o.contacts()
        print(f"scene {k}: {e.n_clumps} clumps, {e.n_spheres} spheres, {len(co['a'])} contacts "
              f"({int((co['b'] >= e.n_spheres).sum())} on the funnel and plate)", flush=True)
        assert len(co["a"]) > e.n_clumps // 2 and (co["b"] >= e.n_spheres).sum() > 10
        compare_pairs(cg, co)
        for key in ("delta", "F", "u", "Ta", "Tb"):
            assert np.array_equal(cg[key], co[key]), (int(k), key)
        sc.step(99)
        o.step(100)
        sg, so = sc.state(), o.state()
        sc.close()
        for key in ("x", "q", "v", "w"):
            assert np.array_equal(sg[key], so[key]), (int(k), key)
