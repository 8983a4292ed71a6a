"""Energy to solution: socket power sampled during a GPU run integrates to a
positive energy and a plausible mean power, in line with the board energy
counter when it advances inside the run (skipped, with the reason, if AMD
SMI cannot be used in this process)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_energy_meter_measures_a_run():
    import paper_1709_09713_amd as ns
    from paper_1709_09713_amd.energy import EnergyMeter
    meter = EnergyMeter()
    if not meter.available:
        pytest.skip(f"AMD SMI energy counter unavailable: {meter.reason}")
    s = ns.Solver(128).init_tgv()
    m = meter.measure(lambda: s.step(1e-3, 100), min_seconds=2.5)
    print(f"energy: {m}", flush=True)
    assert m["seconds"] >= 2.5 and m["calls"] >= 1 and m["joules"] > 0
    assert m["samples"] > 50
    assert 20.0 < m["mean_watts"] < 3000.0
    if m["counter_watts"] is not None:
        assert 0.5 < m["counter_watts"] / m["mean_watts"] < 2.0
    torch.cuda.synchronize()
