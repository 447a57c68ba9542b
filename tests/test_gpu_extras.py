"""GPU checks of the autotuner, the standalone peak selection and the phase entropy on every plan kind."""
import os

import numpy as np
import pytest

import oracle
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


FREQS = np.linspace(0.05, 12.0, 2500)


def test_autotuned_plan_matches_default_and_caches(tmp_path):
    """Launch shapes change only the schedule: the periodogram and peaks are bit-identical."""
    _say("autotune")
    b = synth.random_batch(71, 40, 50, 600, FREQS, 20)
    cache = str(tmp_path / "tune.txt")
    p0 = fpw.Plan.from_batch(b, topk=5)
    p1 = fpw.Plan.from_batch(b, topk=5, autotune=True, tune_cache=cache)
    assert p1.info().tuned == 1 and os.path.exists(cache)
    S0, i0, v0 = p0.eval()
    S1, i1, v1 = p1.eval()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S1.cpu().numpy(), S0.cpu().numpy())
    np.testing.assert_array_equal(i1.cpu().numpy(), i0.cpu().numpy())
    np.testing.assert_array_equal(v1.cpu().numpy(), v0.cpu().numpy())
    # a second plan of the same shape takes the cached choice
    p2 = fpw.Plan.from_batch(b, topk=5, autotune=True, tune_cache=cache)
    i2 = p1.info()
    assert p2.info().tuned == 1
    assert (p2.info().freqs_per_lane, p2.info().chunk_freqs) == (i2.freqs_per_lane, i2.chunk_freqs)
    for p in (p0, p1, p2):
        p.close()


@pytest.mark.parametrize("k,fuse", [(1, 0), (5, 0), (16, 0), (5, -1), (16, -1)])
def test_standalone_topk_matches_fused(k, fuse):
    """fpw_topk over a stored periodogram equals the fused selection and the peak rule (fused pass
    of this small plan, and the three-kernel pass)."""
    _say(f"standalone top-k k={k} fuse_prepare={fuse}")
    b = synth.random_batch(72, 25, 1, 400, FREQS, 12)
    plan = fpw.Plan.from_batch(b, topk=k, fuse_prepare=fuse)
    S, idx, val = plan.eval()
    i2, v2 = plan.topk(S, k)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(i2.cpu().numpy(), idx.cpu().numpy())
    np.testing.assert_array_equal(v2.cpu().numpy(), val.cpu().numpy())
    parity.assert_topk_matches_rule(S.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), k)
    plan.close()


def _entropy_check(plan, t_of_curve, n_bins, idx, freqs):
    H, E, V = plan.phase_entropy(idx)
    torch.cuda.synchronize()
    H, E, V, idx = H.cpu().numpy(), E.cpu().numpy(), V.cpu().numpy(), idx.cpu().numpy()
    for c in range(idx.shape[0]):
        tau = t_of_curve(c)
        for r in range(idx.shape[1]):
            if idx[c, r] < 0:
                assert np.isnan(H[c, r])
                continue
            f = freqs[idx[c, r]]
            if np.any(oracle.edge_distance(tau, f, n_bins) < parity.EPS_BIN):
                continue
            assert abs(H[c, r] - oracle.phase_entropy(tau, f, n_bins)) < 2e-6
            assert abs(E[c, r] - oracle.entropy_expectation(n_bins, len(tau))) < 2e-6
            assert abs(V[c, r] - oracle.entropy_variance(n_bins, len(tau))) < 1e-6 * max(1.0, V[c, r])


def test_phase_entropy_on_shared_and_baseline_plans():
    _say("phase entropy on shared and baseline plans")
    f = synth.random_shared_batch(73, 18, 150, FREQS, 16)
    t, y, dy = f.as_shared()
    ps = fpw.Plan.shared(t, y, dy, f.freqs, 16, topk=4)
    _, idx, _ = ps.eval()
    _entropy_check(ps, lambda c: t, 16, idx, f.freqs)
    ps.close()
    b = synth.random_batch(74, 12, 5, 300, FREQS, 10)
    pb = fpw.Plan.from_batch(b, topk=3, baseline_terms=2)
    _, idx, _ = pb.eval()
    _entropy_check(pb, lambda c: b.curve(c)[0], 10, idx, b.freqs)
    pb.close()


def test_c_client_runs_a_pass(tmp_path):
    """A plain-C program plans, runs a pass through the C ABI and finds the injected period."""
    _say("C client pass")
    import subprocess

    from tests.test_abi import _build_c_client

    exe = _build_c_client(tmp_path)
    r = subprocess.run([exe, "gpu"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "gpu pass ok" in r.stdout


def test_graph_cache_with_alternating_and_many_output_buffers():
    """Captured passes are kept per output buffer set (a few, least recently used dropped):
    replays into alternating and into more buffer sets than are kept all match a direct pass."""
    _say("graph cache")
    b = synth.random_batch(75, 30, 20, 300, FREQS, 16)
    # (three-kernel passes: the fused pass of a plan this small is never captured)
    ref_plan = fpw.Plan.from_batch(b, topk=3, use_graph=False, fuse_prepare=-1)
    S0, i0, v0 = ref_plan.eval()
    torch.cuda.synchronize()
    S0, i0, v0 = S0.cpu().numpy(), i0.cpu().numpy(), v0.cpu().numpy()
    plan = fpw.Plan.from_batch(b, topk=3, fuse_prepare=-1)
    bufs = [(torch.empty_like(torch.from_numpy(S0)).cuda(), torch.empty((b.n_curves, 3), dtype=torch.int32, device="cuda"),
             torch.empty((b.n_curves, 3), dtype=torch.float32, device="cuda")) for _ in range(6)]
    order = [0, 1, 0, 1, 2, 3, 4, 5, 0, 5, 1]
    for j in order:
        S, idx, val = bufs[j]
        S.fill_(-1.0)
        plan.eval(S_out=S, idx_out=idx, val_out=val)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(S.cpu().numpy(), S0)
        np.testing.assert_array_equal(idx.cpu().numpy(), i0)
        np.testing.assert_array_equal(val.cpu().numpy(), v0)
        torch.ones(100, device="cuda").sum().item()  # eager work between replays
    plan.close()
    ref_plan.close()
