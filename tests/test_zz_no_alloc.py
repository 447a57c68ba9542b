"""GPU: fpw_eval_static, the pass that allocates nothing, against fpw_plan + fpw_eval_batch.

The same batch goes through both entry points (the plan folding in the
listing order, as the static pass does, so the bins are the same); S must
agree to the parity bar, and with the oracle; the peaks must follow the
peak rule on the static pass's own S and match the plan's.  Two calls in a
row, the second on a smaller batch, show that the static array's leftovers
from the first call do not leak into the second.  A curve whose weights
exceed the wide format's bound comes back as NaN with no peaks.
"""
import numpy as np
import pytest

from paper_2502_00243_amd import synth
from tests import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU runs deselect this module with -m "not gpu"
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]
else:
    from paper_2502_00243_amd import fpw


def _say(msg):
    print(msg, flush=True)


def _device(b):
    cuda = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()  # noqa: E731
    return (cuda(b.offsets, np.int64), cuda(b.t, np.float64), cuda(b.y, np.float64), cuda(b.dy, np.float64),
            cuda(b.freqs, np.float64))


def _check_against_plan_and_oracle(b, M, k, opts):
    off, t, y, dy, f = _device(b)
    S, idx, val = fpw.eval_static(off, t, y, dy, f, M, topk=k, **opts)
    torch.cuda.synchronize()
    S, idx, val = S.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    plan = fpw.Plan.from_batch(b, n_bins=M, topk=k, phase="fp64_listing", **opts)
    Sp, ip, vp = plan.eval()
    torch.cuda.synchronize()
    Sp, ip, vp = Sp.cpu().numpy(), ip.cpu().numpy(), vp.cpu().numpy()
    plan.close()
    opt = parity.oracle_options(**opts)
    for c in range(b.n_curves):
        tc, yc, dyc = b.curve(c)
        S_ref, S_abs, _ = parity.reference_for_curve(tc, yc, dyc, b.freqs, M, opt)
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"static vs oracle, curve {c}")
        # the existing entry point, same bins: the parity bar between the two
        parity.assert_s_close(S[c], Sp[c].astype(np.float64), S_abs, what=f"static vs plan, curve {c}")
    parity.assert_topk_matches_rule(S, idx, val, k)
    # peaks equal the plan's wherever the two S agree to the last bit, and up to near-ties elsewhere
    for c in range(b.n_curves):
        S_ref = Sp[c].astype(np.float64)
        parity.assert_topk_near_oracle(S_ref, idx[c], val[c], k)
    return S


def test_static_pass_matches_the_plan_twice_in_a_row():
    _say("static pass: 12 ragged curves x 477 freqs, M = 20, top-4; then 5 curves x 200 freqs, M = 7, top-2")
    b1 = synth.random_batch(71, 12, 1, 300, np.linspace(0.05, 30.0, 477), 20)
    _check_against_plan_and_oracle(b1, 20, 4, {})
    b2 = synth.random_batch(72, 5, 1, 120, np.linspace(0.1, 9.0, 200), 7)
    _check_against_plan_and_oracle(b2, 7, 2, dict(center="mean", tref="first", inv_alpha2=30.0))


def test_static_pass_flags_weights_beyond_the_wide_format():
    _say("static pass: a curve with errors over nine decades")
    freqs = np.linspace(0.1, 10.0, 300)
    b = synth.random_batch(73, 4, 50, 200, freqs, 10)
    dy = b.dy.copy()
    a, e = int(b.offsets[2]), int(b.offsets[3])
    dy[a:e] = 10.0 ** np.linspace(-9.0, 0.0, e - a)
    b = synth.Batch(offsets=b.offsets, t=b.t, y=b.y, dy=dy, freqs=freqs, n_bins=10, name="wide range")
    off, t, y, dyd, f = _device(b)
    S, idx, val = fpw.eval_static(off, t, y, dyd, f, 10, topk=3)
    torch.cuda.synchronize()
    S, idx = S.cpu().numpy(), idx.cpu().numpy()
    assert np.all(np.isnan(S[2])) and np.all(idx[2] == -1)
    for c in (0, 1, 3):
        assert np.all(np.isfinite(S[c]))
        S_ref, S_abs, _ = parity.reference_for_curve(*b.curve(c), freqs, 10, parity.oracle_options())
        parity.assert_s_close(S[c], S_ref, S_abs, what=f"curve {c}")


def test_static_pass_refuses_what_its_scratch_cannot_hold():
    # 1e6 points need 32 MB of wide records: beyond the 16 MiB static array, refused before any launch
    n = 1_000_000
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    t = torch.linspace(0, 100, n, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    dy = torch.full((n,), 0.1, dtype=torch.float64, device="cuda")
    f = torch.linspace(0.1, 1.0, 10, dtype=torch.float64, device="cuda")
    with pytest.raises(fpw.FpwError) as e:
        fpw.eval_static(off, t, y, dy, f, 10)
    assert e.value.status == fpw.EUNSUPPORTED
