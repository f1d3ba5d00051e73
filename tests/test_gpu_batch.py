"""The batched form (hpt_run_batch): independent runs advanced concurrently on
their own streams give exactly the trajectories of the same runs advanced one
at a time, and a batched run matches the CPU oracle."""

import pytest

from paper_2606_30985_amd import inputs
from tests.gpu_util import load_hpt

pytestmark = pytest.mark.gpu


def _runs(n, chi, steps_cap):
    out = []
    for r in inputs.batched_runs()[:n]:
        out.append((dict(Lx=r["Lx"], Ly=r["Ly"], J=r["J"], h=r["h"], dt=r["dt"], chi_max=chi),
                    min(r["nsteps"], steps_cap)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_one_at_a_time(precision):
    import torch
    hpt = load_hpt()
    runs = _runs(8, 8, 12)
    solo = []
    for cfg, n in runs:
        s = hpt.Simulator(precision=precision, **cfg)
        traj = []
        for _ in range(n):
            s.step(1)
            traj.append(s.measure())
        s.close()
        solo.append(traj)
    sims = [hpt.Simulator(precision=precision, stream=torch.cuda.Stream(), **cfg) for cfg, _ in runs]
    got = hpt.run_batch(sims, [n for _, n in runs])
    for s in sims:
        s.close()
    for a, b in zip(solo, got):
        assert len(a) == len(b)
        for x, y in zip(a, b):
            assert x["C"] == y["C"] and x["step"] == y["step"] and x["chi_live_max"] == y["chi_live_max"]


def test_batched_run_matches_oracle():
    import torch
    from oracle.network import Config
    from oracle.run import run
    hpt = load_hpt()
    runs = [r for r in _runs(64, 8, 10) if r[0]["Lx"] == 3][:2]
    sims = [hpt.Simulator(precision="fp64", stream=torch.cuda.Stream(), **cfg) for cfg, _ in runs]
    got = hpt.run_batch(sims, [n for _, n in runs])
    for s in sims:
        s.close()
    for (cfg, n), traj in zip(runs, got):
        ref = run(Config(**cfg), n)[0]
        for k in range(n):
            assert abs(traj[k]["C"] - ref[k + 1]["C"]) <= 1e-10, (cfg, k)


def test_batch_rejects_repeated_handles():
    hpt = load_hpt()
    s = hpt.Simulator(Lx=3, Ly=3, chi_max=4)
    with pytest.raises(hpt.HptError):
        hpt.run_batch([s, s], [1, 1])
    s.close()
