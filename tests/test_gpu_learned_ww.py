"""The learned weight-window pipeline on the GPU: pilots, network training
and BF16 inference, windows; the windowed run stays unbiased against analog
and lowers the detector's relative error per history."""
import math

import pytest

import workloads as w


@pytest.mark.gpu
def test_learned_windows_unbiased_and_effective():
    from paper_2305_07636_amd import learned_ww as lw

    p = w.cfg5_dogleg(detector=w.CORNER_DETECTOR)
    table, info = lw.learned_windows(p, n_pilot=2_000_000, steps=800)
    print(f"[lww] n_train {info['n_train']} loss {info['loss_first']:.3g} -> {info['loss_last']:.3g}", flush=True)
    assert info["loss_last"] < 0.2 * info["loss_first"]
    assert (table > 0).sum() > 100
    a = lw.figure_of_merit(p, 20_000_000, 7)
    b = lw.figure_of_merit(p, 2_000_000, 8, table=table)
    print(f"[lww] analog {a}\n[lww] learned {b}", flush=True)
    assert a["mean"] > 0 and b["mean"] > 0
    d = abs(a["mean"] - b["mean"]) / math.hypot(a["sigma"], b["sigma"])
    assert d < 4.0, d
    # relative error per history: windows win
    assert b["R"] ** 2 * 2_000_000 < a["R"] ** 2 * 20_000_000
