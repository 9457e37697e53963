"""GPU tests of the batched multi-system launch: parity with the single-system
path and the oracle, graph capture and replay, the autotuner, and the
network-fed variant."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import assert_eloc_close, dev, eloc_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


# uneven systems: N = 16 .. 120 (one- and two-word keys), ragged sample counts
SYSTEMS = [dict(K=8, n_up=2, n_dn=2, n_unique=300), dict(K=12, n_up=4, n_dn=3, n_unique=1000),
           dict(K=24, n_up=6, n_dn=6, n_unique=3001), dict(K=40, n_up=5, n_dn=6, n_unique=777),
           dict(K=60, n_up=5, n_dn=5, n_unique=129)]


def _items(nn, specs, with_model=False):
    items = []
    for k, kw in enumerate(specs):
        d = synth.config_inputs(2, sys=k, model=with_model, **kw)
        n = d["keys"].shape[0]
        S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
        it = dict(d=d, system=S, table=nn.Table(S, capacity=n), keys=dev(d["keys"]),
                  counts=dev(d["counts"], torch.int32), logabs=dev(d["logabs"]), phase=dev(d["phase"]),
                  eloc=torch.full((n, 2), np.nan, dtype=torch.float64, device="cuda"),
                  energy=torch.zeros(4, dtype=torch.float64, device="cuda"))
        if with_model:
            it["model"] = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
        items.append(it)
    return items


def _single(nn, it):
    """The same system through the single-system entry points."""
    T = nn.Table(it["system"], capacity=it["keys"].shape[0])
    T.build(it["keys"], it["logabs"], it["phase"], validate=True)
    return nn.eloc_table(it["system"], T, it["keys"], it["counts"], it["logabs"], it["phase"])


def test_batch_matches_single_system_and_oracle(nn):
    _print_case("batch_parity", systems=len(SYSTEMS))
    items = _items(nn, SYSTEMS)
    B = nn.Batch(items)
    B.run()
    torch.cuda.synchronize()
    for it in items:
        e1, en1 = _single(nn, it)
        torch.cuda.synchronize()
        a, b = eloc_complex(it["eloc"]), eloc_complex(e1)
        assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(1.0, np.abs(b))), it["d"]["K"]
        assert abs(it["energy"][0].item() - en1[0].item()) <= 1e-12 * abs(en1[0].item())
    # the two smallest systems against the FP64 oracle
    for it in items[:2]:
        d = it["d"]
        ref, ab = oracle.eloc_table(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["keys"],
                                    d["logabs"], d["phase"], d["keys"], d["logabs"], d["phase"], with_absum=True)
        assert_eloc_close(eloc_complex(it["eloc"]), ref, ab, label=f"K={d['K']}")


def test_batch_graph_replays_match_eager(nn):
    _print_case("batch_graph")
    items = _items(nn, SYSTEMS[:4])
    B = nn.Batch(items)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.run(s)
    s.synchronize()
    ref = [it["eloc"].clone() for it in items]
    ref_en = [it["energy"].clone() for it in items]
    B.capture(s)
    for rep in range(3):
        for it in items:  # eager work between replays
            it["eloc"].fill_(np.nan)
            it["energy"].zero_()
        torch.cuda.synchronize()
        B.launch(s)
        s.synchronize()
        for it, r, re in zip(items, ref, ref_en):
            assert torch.equal(it["eloc"], r), rep
            assert torch.equal(it["energy"], re), rep


def test_batch_autotune_keeps_results(nn):
    _print_case("batch_autotune")
    items = _items(nn, SYSTEMS[1:4])
    B = nn.Batch(items)
    B.run()
    torch.cuda.synchronize()
    ref = [eloc_complex(it["eloc"]) for it in items]
    tune, ms = B.autotune(reps=1)
    print(f"autotuned schedule {tune}, {ms:.3f} ms per step")
    assert tune["waves_per_block"] in (8, 12) and tune["search"] in (1, 2)
    assert tune["tile_samples"] in (64, 256, 1024) and tune["splitter_levels"] in (8, 10, 12)
    assert B.get_tune() == tune
    for it in items:
        it["eloc"].fill_(np.nan)
    B.run()
    torch.cuda.synchronize()
    for it, r in zip(items, ref):
        g = eloc_complex(it["eloc"])
        assert np.all(np.abs(g - r) <= 1e-12 * np.maximum(1.0, np.abs(r)))


def test_batch_autotune_cache_round_trip(nn, tmp_path):
    """A batch schedule timed once is stored under the batch's key (device,
    item count, digest of the items' workload keys) and used again by an
    equal batch without timing; results are unchanged."""
    _print_case("batch_autotune_cache")
    path = str(tmp_path / "tune.txt")
    items = _items(nn, SYSTEMS[1:3])
    B = nn.Batch(items)
    key = B.tune_key()
    assert ":batch2:" in key and key.startswith("gfx")
    tune, ms = B.autotune(reps=1, cache_path=path)
    assert nn.tune_cache_lookup(path, key) == (tune, pytest.approx(ms))
    B.run()
    torch.cuda.synchronize()
    ref = [it["eloc"].clone() for it in items]
    items2 = _items(nn, SYSTEMS[1:3])
    B2 = nn.Batch(items2)
    assert B2.tune_key() == key
    tune2, ms2 = B2.autotune(reps=1, cache_path=path)
    assert tune2 == tune and ms2 == pytest.approx(ms) and B2.get_tune() == tune
    B2.run()
    torch.cuda.synchronize()
    for it, r in zip(items2, ref):
        assert torch.equal(it["eloc"], r)
    assert nn.Batch(_items(nn, SYSTEMS[2:4])).tune_key() != key


def test_batch_with_models_feeds_the_table_from_the_network(nn):
    _print_case("batch_models")
    specs = [dict(K=6, n_up=2, n_dn=3, n_unique=150), dict(K=12, n_up=3, n_dn=3, n_unique=700),
             dict(K=20, n_up=4, n_dn=4, n_unique=333)]
    items = _items(nn, specs, with_model=True)
    B = nn.Batch(items)
    B.run()
    torch.cuda.synchronize()
    for it in items:
        la, ph = nn.model_logpsi(it["model"], it["keys"], nn.NNQS_BF16)
        torch.cuda.synchronize()
        assert torch.equal(la, it["logabs"]) and torch.equal(ph, it["phase"])
        e1, en1 = _single(nn, it)
        torch.cuda.synchronize()
        a, b = eloc_complex(it["eloc"]), eloc_complex(e1)
        assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(1.0, np.abs(b)))


def test_batch_rejects_bad_items(nn):
    items = _items(nn, SYSTEMS[:1])
    bad = dict(items[0])
    bad["table"] = nn.Table(bad["system"], capacity=10)  # smaller than n
    with pytest.raises(nn.NNQSError):
        nn.Batch([bad])
    B = nn.Batch(items)
    with pytest.raises(nn.NNQSError):  # nothing captured yet
        B.launch(torch.cuda.Stream())
    with pytest.raises(nn.NNQSError):
        B.set_tune(search=3)


MODEL_SYSTEMS = [dict(K=4, n_up=2, n_dn=2, n_unique=30), dict(K=8, n_up=2, n_dn=2, n_unique=50),
                 dict(K=12, n_up=4, n_dn=3, n_unique=40), dict(K=20, n_up=7, n_dn=7, n_unique=6),
                 dict(K=33, n_up=5, n_dn=6, n_unique=3)]


def test_batch_model_matches_single_system_and_oracle(nn):
    """Batched transformer mode: five systems (N = 8 .. 66, one- and two-word
    keys) whose connections go through one persistent launch of the
    prefix-reusing BF16 forward.  Each item equals the single-system BF16
    full path exactly (same kernels per configuration), graph replays are
    checked against the eager step, and the two smallest systems are within
    the BF16 error of the FP64 oracle."""
    _print_case("batch_model", systems=len(MODEL_SYSTEMS))
    items = []
    for k, kw in enumerate(MODEL_SYSTEMS):
        d = synth.config_inputs(2, sys=10 + k, model=True, **kw)
        n = d["keys"].shape[0]
        S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
        items.append(dict(d=d, system=S, model=nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"]),
                          keys=dev(d["keys"]), counts=dev(d["counts"], torch.int32),
                          eloc=torch.full((n, 2), np.nan, dtype=torch.float64, device="cuda"),
                          energy=torch.zeros(4, dtype=torch.float64, device="cuda")))
    B = nn.BatchModel(items)
    B.run()
    torch.cuda.synchronize()
    eager = [(it["eloc"].clone(), it["energy"].clone()) for it in items]
    for it, (e, en) in zip(items, eager):
        e1, en1, _ = nn.eloc_model(it["system"], it["model"], it["keys"], it["counts"], nn.NNQS_BF16)
        torch.cuda.synchronize()
        assert torch.equal(e, e1), it["d"]["K"]
        assert torch.equal(en, en1), it["d"]["K"]
    st = torch.cuda.Stream()
    B.capture(st)
    for rep in range(3):
        for it in items:
            it["eloc"].fill_(np.nan)
        torch.cuda.synchronize()
        B.launch(st)
        st.synchronize()
        for it, (e, en) in zip(items, eager):
            assert torch.equal(it["eloc"], e), (rep, it["d"]["K"])
            assert torch.equal(it["energy"], en), (rep, it["d"]["K"])
        torch.zeros(1024, device="cuda").sum().item()  # eager work between replays
    for it in items[:2]:
        d = it["d"]
        ora, absum = oracle.eloc_model(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["weights"],
                                       d["model_shape"], d["keys"], with_absum=True)
        g = eloc_complex(it["eloc"])
        rel = np.abs(g - ora) / absum
        print(f"batch model K={d['K']}: BF16 vs FP64 oracle max |dE|/A {rel.max():.3e}")
        assert rel.max() <= 0.05
