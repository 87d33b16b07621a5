"""The benchmark's command-line contract, checked without a GPU."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_pass_kernel_names():
    from paper_2001_11220_amd import etd
    e = etd.EtdRdp((256, 256, 256), ("periodic",) * 3, (2e-5, 1e-5), 1.0, "gray_scott",
                   {"F": 0.04, "kappa": 0.06})
    assert [e.pass_kernel(p) for p in (1, 2, 3)] == ["k_first_pair<8, 16, 2, true, false, double>",
                                                      "k_mid_s<8, 2, 32, 2, true, double>",
                                                      "k_last_s<8, 2, 32, 2, true, double>"]
    f = etd.EtdRdp((512, 512, 512), ("dirichlet",) * 3, (1.0, 10.0), 1e-4, "schnakenberg",
                   {"a": 0.1, "b": 0.9, "gamma": 1.0})
    assert [f.pass_kernel(p) for p in (1, 2, 3)] == ["k_first_s<8, 2, 16, 1, true, false, double>",
                                                      "k_mid_s<8, 2, 16, 1, true, double>",
                                                      "k_last_s<8, 2, 16, 1, true, double>"]
    one = etd.EtdRdp((256, 256, 256), ("periodic",) * 3, (2e-5, 1e-5), 1.0, "gray_scott",
                     {"F": 0.04, "kappa": 0.06}, lines_per_wave=1)
    assert [one.pass_kernel(p) for p in (1, 2, 3)] == ["k_first<4, 2, 16, true, double>", "k_mid<4, 2, 16, true, double>",
                                                        "k_last<4, 2, 16, true, double>"]
    g = etd.EtdRdp((320, 64), ("neumann",) * 2, (0.1,), 0.1, "linear", {"C": [[-1.0]]})
    assert [g.pass_kernel(p) for p in (1, 2)] == ["k_first<5, 1, 8, false, double>", "k_last<1, 1, 16, false, double>"]
    import pytest
    with pytest.raises(etd.EtdError):
        g.pass_kernel(3)
    sys.path.insert(0, ROOT)
    import bench
    assert bench.pass_names(e, 3) == [e.pass_kernel(p) for p in (1, 2, 3)]
    assert bench.pass_words(3) == [4, 6, 4] and bench.pass_words(2) == [4, 4]


def test_precision_option_is_refused_where_not_built():
    for wl in ("schnakenberg3d_adjoint", "cgl3d_complex"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", wl,
                            "--precision", "f32"], capture_output=True, text=True, timeout=120)
        assert r.returncode == 2, (wl, r.stderr)
        assert r.stdout.strip() == ""


def test_unknown_workload_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "unknown workload" in r.stderr
    assert r.stdout.strip() == ""


def test_pooled_oracle_equals_the_plain_oracle():
    """The all-core timing of cpu_baseline spreads the oracle's own line
    routines over worker processes; the step it computes is the same."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import oracle as O
    from paper_2001_11220_amd import workloads as W

    prob = W.grayscott3d(shape=(12, 10, 8))
    prob.bcs = ("periodic", "neumann", "dirichlet")
    u = prob.initial()
    lam = np.random.default_rng(2).standard_normal(u.shape)
    ref = O.etd_rdp_if_step(u, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.params)
    aref = O.adjoint_step(u, lam, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.params)
    pool = bench.OraclePool(3, u.nbytes)
    try:
        with pool:
            got = O.etd_rdp_if_step(u, prob.k, prob.D, prob.bcs, prob.hs(), prob.model, prob.params)
            agot = O.adjoint_step(u, lam, prob.k, prob.D, prob.bcs, prob.hs(), prob.model,
                                  prob.params)
        assert O.etd_rdp_oracle.solve_axis is bench._POOL["orig"]["solve_axis"]
    finally:
        pool.close()
    assert np.array_equal(got, ref)
    assert np.array_equal(agot[0], aref[0])
    assert np.allclose(agot[1], aref[1], rtol=1e-13) and np.allclose(agot[2], aref[2], rtol=1e-13)
