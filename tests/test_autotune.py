"""The tuning sweep's selection logic, on a stand-in solver whose step cost
is a known function of the settings plus a drift (no GPU)."""
from paper_2607_09552_amd import autotune


class _Fake:
    def __init__(self):
        self.cfg = dict(batch_steps=32, use_graph=1, transport_block=256, shakhov_lanes=4, scatter_block=512,
                        tally_block=256, flux_block=256)
        self.t = 0.0
        self.n = 0

    def tuning(self):
        return dict(self.cfg)

    def set_tuning(self, **kw):
        assert set(kw) <= set(self.cfg)
        self.cfg.update(kw)

    def work(self):
        return self.n

    def step(self, k):
        c = self.cfg
        cost = 1.0 + 0.01 * abs(c["batch_steps"] - 16) + 0.05 * (1 - c["use_graph"]) \
            + 0.02 * (c["transport_block"] != 128) + 0.03 * abs(c["shakhov_lanes"] - 8) / 4 \
            + 0.02 * (c["scatter_block"] != 128) + 0.015 * (c["tally_block"] != 64) + 0.01 * (c["flux_block"] != 256)
        self.t += k * cost * (1.0 + 1e-4 * self.n / 1000.0)  # the flow slowly gets more expensive
        self.n += k * 1000


def test_sweep_finds_the_cheapest_settings_despite_drift():
    f = _Fake()
    best, table = autotune.sweep(f, rounds=5, steps=16, log=lambda m: None, clock=lambda: f.t, sync=lambda: None)
    assert best == dict(batch_steps=16, use_graph=1, transport_block=128, shakhov_lanes=8, scatter_block=128,
                        tally_block=64, flux_block=256)
    assert f.cfg == best
    assert len(table) >= 4


class _FakeFlat(_Fake):
    """Only two settings matter: a transport block of 128 saves 2 %, a tally
    block of 64 saves 0.1 % (less than the sweep's noise threshold)."""

    def step(self, k):
        c = self.cfg
        cost = 1.0 - 0.02 * (c["transport_block"] == 128) - 0.001 * (c["tally_block"] == 64)
        self.t += k * cost
        self.n += k * 1000


def test_sweep_keeps_the_current_value_within_the_noise():
    f = _FakeFlat()
    best, _ = autotune.sweep(f, rounds=5, steps=16, log=lambda m: None, clock=lambda: f.t, sync=lambda: None)
    assert best["transport_block"] == 128
    assert best["tally_block"] == 256 and best == dict(f.tuning())


def test_load_tuning_missing_file(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "TUNING_FILE", str(tmp_path / "none.json"))
    assert autotune.load_tuning("cylinder") is None
