"""Ensemble kernel forms and the autotuner: every form the tuner may pick for
a (group, pass) is parity-green against the oracle, in FP64 and FP32 and for
both schemes; the tuner leaves the state advanced by one step of its plan;
cached plans are reused."""

import numpy as np
import pytest

import oracle as O
from paper_2001_11220_amd import workloads as W

pytestmark = pytest.mark.gpu

# groups with lines of 32 m rows (all three forms), chunks of 3-8 rows
# (streamed) and short or odd lines (unsplit only), every boundary condition
SIZES = (40, 64, 96, 128, 160, 192, 224, 256, 288, 320, 384, 448, 512)


def ensemble(prec_seed=0):
    ens = W.brusselator_ensemble(ninst=30, nsteps=2, seed=11 + prec_seed, sizes=SIZES)
    rng = np.random.default_rng(5 + prec_seed)
    for ins in ens.instances:  # some non-square grids and Dirichlet axes too
        if rng.random() < 0.3:
            ins["shape"] = (ins["shape"][0], int(rng.choice(SIZES)))
        ins["bcs"] = tuple(str(rng.choice(["neumann", "periodic", "dirichlet"])) for _ in range(2))
    ens.states = [0.5 + 0.1 * rng.random((2, ins["shape"][1], ins["shape"][0])) for ins in ens.instances]
    return ens


def oracle_steps(ens, i, nsteps, scheme="rdp"):
    ins = ens.instances[i]
    hs = [O.default_h(n, bc) for n, bc in zip(ins["shape"], ins["bcs"])]
    step = O.etd1_if_step if scheme == "etd1" else O.etd_rdp_if_step
    u = ens.states[i]
    for _ in range(nsteps):
        u = step(u, ens.k, ins["D"], ins["bcs"], hs, ens.model, ins["params"])
    return u


def check(b, u, ens, nsteps, tol, scheme="rdp", label=""):
    worst = 0.0
    for i in range(b.n):
        got = b.view(u, i).cpu().numpy().astype(np.float64)
        ref = oracle_steps(ens, i, nsteps, scheme)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        em = float(np.abs(got - ref).max() / np.abs(ref).max())
        worst = max(worst, err, em)
        assert err <= tol and em <= tol, (label, i, ens.instances[i]["shape"], err, em)
    print(f"[forms] {label} worst={worst:.2e}", flush=True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["rdp", "etd1"])
def test_every_form_matches_oracle(prec, scheme):
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = ensemble(1 if prec == "f32" else 0)
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k, precision=prec, scheme=scheme)
    groups = b.groups()
    default = b.plan
    tol = 1e-12 if prec == "f64" else 2e-5
    for form in (0, 1, 2):
        plan = [form if b.form_allowed(g, p, form) else default[2 * g + p]
                for g in range(len(groups)) for p in range(2)]
        b.plan = plan
        assert b.plan == plan
        u = b.pack(ens.states)
        b.step(u, 2, use_graph=True)
        torch.cuda.synchronize()
        check(b, u, ens, 2, tol, scheme, f"{prec} {scheme} form {form} plan {plan}")
    b.close()


def test_tuner_advances_one_step_and_keeps_a_valid_plan(tmp_path):
    import torch
    from paper_2001_11220_amd import tuning
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = ensemble()
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    u = b.pack(ens.states)
    times = b.tune(u, reps=2)
    torch.cuda.synchronize()
    plan = b.plan
    for g in range(len(b.groups())):
        for p in range(2):
            assert b.form_allowed(g, p, plan[2 * g + p])
            t = times[g][p]
            assert t[plan[2 * g + p]] == min(v for v in t if v is not None)
    check(b, u, ens, 1, 1e-12, label="after tune")
    b.step(u, 1, use_graph=True)  # the tuned plan, in a graph
    torch.cuda.synchronize()
    check(b, u, ens, 2, 1e-12, label="tuned plan")
    # the cache: a second ensemble of the same layout takes the stored plan
    path = str(tmp_path / "plans.json")
    u2 = b.pack(ens.states)
    plan1, t1 = tuning.tune_batch(b, u2, reps=2, path=path)
    assert t1 is not None
    c = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    u3 = c.pack(ens.states)
    plan2, t2 = tuning.tune_batch(c, u3, path=path)
    assert t2 is None and plan2 == plan1 and c.plan == plan1
    b.close()
    c.close()


def test_group_pass_entry_runs_one_group():
    import torch
    from paper_2001_11220_amd.etd import EtdRdpBatch
    ens = ensemble()
    b = EtdRdpBatch(ens.instances, ens.s, ens.model, ens.k)
    u = b.pack(ens.states)
    for p in range(2):
        for g in range(len(b.groups())):
            b.group_pass(u, g, p)
    torch.cuda.synchronize()
    check(b, u, ens, 1, 1e-12, label="group by group")
    b.close()
