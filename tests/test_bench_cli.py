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
    assert [e.pass_kernel(p) for p in (1, 2, 3)] == ["k_first_s<8, 2, 32, 2, true, false, double>",
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
