"""Scheduling logic of the serving loop, on the CPU with fake slots (no GPU).

The fake slot fits a batch with the CPU oracle and reports completion after a fixed delay, so
admission by memory, FIFO batching, continuous batching over several slots, per-event results
and latency bookkeeping can be checked without a device.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1312_0917_amd import serve, synth


class FakeSlot:
    def __init__(self, bank, cap_words, delay_s, clock):
        self.bank, self.cap, self.delay, self.clock = bank, cap_words, delay_s, clock
        self.t_launch = None
        self.launched = []
        self.retries = 0

    def fits(self, n_words, n_events):
        return n_words <= self.cap

    def launch(self, words, e0, e1):
        assert len(words) <= self.cap
        self.t_launch = self.clock()
        self.launched.append((e0, e1))
        self.res = oracle.run(words, self.bank.f, self.bank.q, oracle.make_config(), combos=False)
        self.n = e1 - e0

    def poll(self):
        return self.clock() - self.t_launch >= self.delay

    def collect(self):
        r = self.res
        arrays = {k: r["best_" + k] for k in ("nacc", "k", "p0", "p1", "p2", "chi2")}
        arrays["set"] = r["road_set"]
        per_event = serve.split_by_event(r["road_event"], arrays, self.n)
        return r["n_combos"], per_event


@pytest.fixture(scope="module")
def stream_and_bank():
    bank = synth.make_bank()
    s = synth.make_sample("c4", n_events=120, bank=bank)
    arr = synth.poisson_arrivals(s.n_events, rate_hz=20e3, seed=3)
    return serve.EventStream(s.words, s.event_word_begin, arr), s, bank


def test_fifo_batches_cover_every_event_once(stream_and_bank):
    st, s, bank = stream_and_bank
    slots = [FakeSlot(bank, 40000, 2e-3, time.perf_counter) for _ in range(3)]
    stats, res = serve.serve(st, slots, max_events=16, keep_results=True)
    launched = sorted(b for sl in slots for b in sl.launched)
    # consecutive FIFO prefixes: the batches tile [0, n) without gaps or overlaps
    assert launched[0][0] == 0 and launched[-1][1] == st.n_events
    for (a0, a1), (b0, b1) in zip(launched, launched[1:]):
        assert a1 == b0 and a1 > a0
    assert all(b1 - b0 <= 16 for b0, b1 in launched)
    assert max(len(sl.launched) for sl in slots) < len(launched)  # several slots used
    assert np.all(stats.latency_s > 0) and not np.isnan(stats.latency_s).any()
    assert stats.n_combos == s.expected_combos()


def test_admission_respects_slot_memory(stream_and_bank):
    st, s, bank = stream_and_bank
    cap = 6000
    slots = [FakeSlot(bank, cap, 1e-4, time.perf_counter) for _ in range(2)]
    stats, _ = serve.serve(st, slots, max_events=256)
    for sl in slots:
        for e0, e1 in sl.launched:
            assert st.n_words(e0, e1) <= cap


def test_results_alone_equal_results_in_the_mix(stream_and_bank):
    """Each event's best tracks are the same whether it is fitted alone or inside a batch."""
    st, s, bank = stream_and_bank
    slots = [FakeSlot(bank, 40000, 1e-3, time.perf_counter) for _ in range(2)]
    _, res = serve.serve(st, slots, max_events=32, keep_results=True)
    for e in range(0, st.n_events, 7):
        alone = oracle.run(st.slice(e, e + 1), bank.f, bank.q, oracle.make_config(), combos=False)
        for k in ("nacc", "k", "p0", "p1", "p2", "chi2"):
            assert np.array_equal(res[e][k], alone["best_" + k]), (e, k)


def test_latency_includes_waiting_for_a_slot(stream_and_bank):
    """With one slow slot, later events wait: their latency exceeds the service time."""
    st, s, bank = stream_and_bank
    slots = [FakeSlot(bank, 40000, 5e-3, time.perf_counter)]
    stats, _ = serve.serve(st, slots, max_events=8)
    assert stats.latency_s.max() > 5e-3 * 3
    summ = stats.summary()
    assert summ["p99_us"] >= summ["p50_us"] > 0 and summ["events"] == st.n_events


def test_packet_sizes_pick_leading_events():
    from paper_1312_0917_amd import transfer
    ewb = np.array([0, 100, 250, 400, 1000], dtype=np.int64)  # words per event: 100,150,150,600
    assert transfer.packet_events(ewb, 4) == 1
    assert transfer.packet_events(ewb, 400) == 1        # 100 words = 400 bytes
    assert transfer.packet_events(ewb, 404) == 2
    assert transfer.packet_events(ewb, 1600) == 3
    assert transfer.packet_events(ewb, 10**9) == 4      # everything


class TimedFakeSlot(FakeSlot):
    """A fake slot that reports a device time for each batch, as a timing GPU slot does."""

    def collect(self):
        self.last_device_s = self.delay / 2
        return super().collect()


def test_latency_breakdown_adds_up(stream_and_bank):
    """queue + enqueue + device + visible is each event's latency, every part from its batch."""
    st, s, bank = stream_and_bank
    slots = [TimedFakeSlot(bank, 40000, 1e-3, time.perf_counter) for _ in range(2)]
    stats, _ = serve.serve(st, slots, max_events=16)
    total = stats.queue_s + stats.enqueue_s + stats.device_s + stats.visible_s
    assert np.allclose(total, stats.latency_s, rtol=0, atol=1e-9)
    assert np.all(stats.queue_s >= 0) and np.all(stats.enqueue_s >= 0)
    assert np.allclose(stats.device_s, 0.5e-3)
    b = stats.summary()["breakdown"]
    assert set(b) == {"queue", "enqueue", "device", "visible"}
    # slots that time nothing leave the device part out of the breakdown
    plain = serve.serve(st, [FakeSlot(bank, 40000, 1e-3, time.perf_counter)], max_events=16)[0]
    assert np.isnan(plain.device_s).all() and "device" not in plain.summary()["breakdown"]


def test_launch_capacity_is_the_smallest_power_of_two_that_holds_the_batch():
    assert serve.launch_capacity(1, 700000, 4096) == 4096
    assert serve.launch_capacity(4096, 700000, 4096) == 4096
    assert serve.launch_capacity(4097, 700000, 4096) == 8192
    assert serve.launch_capacity(600000, 700000, 4096) == 700000  # capped at the slot
    caps = serve.launch_capacities(700000, 4096)
    assert caps == [4096 << i for i in range(8)] + [700000]
    for n in (1, 5000, 70000, 524288, 524289, 700000):
        assert serve.launch_capacity(n, 700000, 4096) in caps
        assert serve.launch_capacity(n, 700000, 4096) >= n
