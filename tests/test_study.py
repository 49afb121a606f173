"""Host logic of the reconstruction study (Sec. 9): refinement and
restriction indices, the post-processing of eq. (postproc) and the stopping
rule of Algorithm 3.  The GPU run is in tests/test_gpu_study.py."""
import numpy as np

from paper_1509_01399_amd import study


def test_refine_cubes_covers_the_same_region():
    rng = np.random.default_rng(0)
    s = rng.standard_normal((3, 4, 5))
    f = study.refine_cubes(s)
    assert f.shape == (6, 8, 10)
    for z in range(6):
        for y in range(8):
            for x in range(10):
                assert f[z, y, x] == s[z // 2, y // 2, x // 2]


def test_restrict_trace_takes_coarse_nodes_and_levels():
    fine = np.arange(9 * 7 * 7, dtype=float).reshape(9, 7, 7)
    c = study.restrict_trace(fine)
    assert c.shape == (5, 4, 4)
    assert c[2, 1, 3] == fine[4, 2, 6]


def test_postprocess_threshold():
    a = np.array([1.0, 1.2, 2.9, 3.1, 5.0])
    out = study.postprocess(a)
    # 0.6 * 5 = 3: keeps 3.1 and 5, sets the rest to 1
    assert np.array_equal(out, [1.0, 1.0, 1.0, 3.1, 5.0])


def test_stopping_rule():
    assert not study.stabilised([1.0], 0.05)
    assert not study.stabilised([1.0, 0.9], 0.05)
    assert study.stabilised([1.0, 0.96], 0.05)
    assert study.stabilised([1.0, 1.04], 0.05)


def test_add_noise_kinds():
    """Both noise readings: additive noise has standard deviation level *
    max|obs| everywhere; relative noise scales each datum (zero data stay
    zero) with standard deviation level of the ratio."""
    import numpy as np

    from paper_1509_01399_amd import synth
    rng = np.random.default_rng(3)
    obs = rng.standard_normal((40, 50, 50))
    obs[:5] = 0.0
    add = synth.add_noise(obs, 0.03, 1)
    assert abs(np.std(add - obs) / (0.03 * np.max(np.abs(obs))) - 1.0) < 0.02
    rel = synth.add_noise(obs, 0.03, 1, kind="relative")
    assert np.all(rel[:5] == 0.0)
    ratio = rel[5:] / obs[5:]
    assert abs(np.std(ratio - 1.0) / 0.03 - 1.0) < 0.02
    assert np.array_equal(synth.add_noise(obs, 0.0, 1, kind="relative"), obs)
