"""Seeded synthetic light-curve workloads.

This module only draws inputs: observation times, fluxes, flux errors and
trial-frequency grids.  It holds none of the periodogram's arithmetic, so
the CPU oracle and the GPU path can both take their inputs from here.

The survey data the paper works on (ZTF photometry, Secs. 3.1-3.3 and App. C)
is not available; these generators stand in for its shape: nightly sampling
with seasonal gaps, percent-level lognormal errors, hundreds to thousands of
points per source and frequency grids of 1e4-1e6 trial frequencies.

Every workload is a :class:`Batch`: curves are concatenated in CSR form
(``offsets[c]:offsets[c+1]`` indexes curve ``c``), times are sorted
ascending within a curve, and ``labels`` records what was injected.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Batch",
    "workload",
    "single_curve",
    "ztf_batch",
    "uneven_batch",
    "stress_batch",
    "shared_batch",
    "random_batch",
    "random_shared_batch",
    "GRIDS",
]

# Trial-frequency grids (1/day): start, stop, count; and the bin count of each workload.
GRIDS = {
    "single": (0.01, 10.0, 10_000),
    "ztf": (0.05, 50.0, 100_000),
    "uneven": (0.05, 50.0, 200_000),
    "stress": (0.01, 200.0, 1_000_000),
}
BINS = {"single": 10, "ztf": 20, "uneven": 20, "stress": 50}
# independent seed streams per workload
_SEED_ID = {"single": 1, "ztf": 2, "uneven": 4, "stress": 5, "shared": 6}

_KINDS = ("noise", "sinusoid", "eclipse", "sawtooth", "double")


@dataclass
class Batch:
    offsets: np.ndarray  # int64 [n_curves + 1]
    t: np.ndarray  # float64 [n_points], days
    y: np.ndarray  # float64 [n_points], flux
    dy: np.ndarray  # float64 [n_points], 1-sigma flux error
    freqs: np.ndarray  # float64 [n_freq], 1/day
    n_bins: int
    labels: list = field(default_factory=list)  # per curve: dict(kind, f0, ...)
    name: str = ""

    @property
    def n_curves(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_points(self) -> int:
        return int(self.offsets[-1])

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def curve(self, c: int):
        a, b = int(self.offsets[c]), int(self.offsets[c + 1])
        return self.t[a:b], self.y[a:b], self.dy[a:b]

    def as_shared(self):
        """(t [n_points], y [n_curves, n_points], dy [n_curves, n_points]) when every curve has the same times."""
        n = self.lengths
        if not np.all(n == n[0]):
            raise ValueError("curves differ in length")
        t = self.t.reshape(self.n_curves, int(n[0]))
        if not np.array_equal(t, np.broadcast_to(t[0], t.shape)):
            raise ValueError("curves differ in their times")
        return t[0].copy(), self.y.reshape(t.shape).copy(), self.dy.reshape(t.shape).copy()

    def evals(self) -> int:
        """Observation x frequency evaluations one periodogram pass performs."""
        return int(self.n_points) * int(len(self.freqs))

    def subset(self, curves) -> "Batch":
        curves = np.asarray(curves, dtype=np.int64)
        parts_t, parts_y, parts_dy, offs = [], [], [], [0]
        for c in curves:
            t, y, dy = self.curve(int(c))
            parts_t.append(t)
            parts_y.append(y)
            parts_dy.append(dy)
            offs.append(offs[-1] + len(t))
        return Batch(
            offsets=np.asarray(offs, dtype=np.int64),
            t=np.concatenate(parts_t) if parts_t else np.zeros(0),
            y=np.concatenate(parts_y) if parts_y else np.zeros(0),
            dy=np.concatenate(parts_dy) if parts_dy else np.zeros(0),
            freqs=self.freqs,
            n_bins=self.n_bins,
            labels=[self.labels[int(c)] for c in curves] if self.labels else [],
            name=self.name + "[subset]",
        )


def _seed(name: str, n_curves: int):
    ss = np.random.SeedSequence([2502, 243, _SEED_ID[name]])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n_curves)]


def _ztf_sigma(rng, n):
    """Lognormal per-point errors with a 0.02 median, clipped to [0.002, 0.5]."""
    return np.clip(0.02 * np.exp(0.5 * rng.standard_normal(n)), 0.002, 0.5)


def _observable_nights(n_days: float) -> np.ndarray:
    """Integer nights in [0, n_days) outside a 120-day seasonal gap per year."""
    n = np.arange(int(np.ceil(n_days)), dtype=np.float64)
    n = n[n < n_days]
    return n[np.mod(n, 365.25) < 245.25]


def _nightly_times(rng, nights: np.ndarray, n: int, replace: bool) -> np.ndarray:
    """One exposure per chosen night, at 0.15-0.40 day into the night."""
    chosen = rng.choice(nights, size=n, replace=replace)
    t = chosen + 0.15 + 0.25 * rng.random(n)
    return np.sort(t)


def _log_uniform(rng, lo, hi):
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def _waveform(kind: str, phase: np.ndarray, duty: float) -> np.ndarray:
    """Unit-amplitude periodic shapes of the phase in [0, 1)."""
    if kind == "sinusoid":
        return np.sin(2.0 * np.pi * phase)
    if kind == "eclipse":
        return -(phase < duty).astype(np.float64)
    if kind == "sawtooth":
        return phase - 0.5
    if kind == "double":
        return -np.cos(4.0 * np.pi * phase) - 0.3 * np.cos(2.0 * np.pi * phase)
    raise ValueError(kind)


def _signal_to_noise(s: np.ndarray, dy: np.ndarray) -> float:
    """Signal chi-square against a constant: sqrt(sum((s - mean s)^2 / dy^2))."""
    r = (s - s.mean()) / dy
    return float(np.sqrt(np.dot(r, r)))


def _assemble(curves, freqs, n_bins, labels, name) -> Batch:
    offs = np.zeros(len(curves) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(c[0]) for c in curves])
    return Batch(
        offsets=offs,
        t=np.concatenate([c[0] for c in curves]),
        y=np.concatenate([c[1] for c in curves]),
        dy=np.concatenate([c[2] for c in curves]),
        freqs=freqs,
        n_bins=n_bins,
        labels=labels,
        name=name,
    )


def _grid(name: str) -> np.ndarray:
    lo, hi, n = GRIDS[name]
    return np.linspace(lo, hi, n)


def single_curve() -> Batch:
    """One curve: 200 uniform times over 1000 d, a 0.05-amplitude 0.37-d sinusoid."""
    (rng,) = _seed("single", 1)
    n = 200
    t = np.sort(rng.uniform(0.0, 1000.0, n))
    dy = rng.uniform(0.01, 0.05, n)
    y = 0.05 * np.sin(2.0 * np.pi * t / 0.37) + dy * rng.standard_normal(n)
    lab = [dict(kind="sinusoid", f0=1.0 / 0.37, amp=0.05)]
    return _assemble([(t, y, dy)], _grid("single"), BINS["single"], lab, "single_curve")


def ztf_batch(n_curves: int = 1000) -> Batch:
    """ZTF-like cadence over 1500 d: 10% sinusoids, 10% box eclipses, 80% noise."""
    rngs = _seed("ztf", n_curves)
    nights = _observable_nights(1500.0)
    curves, labels = [], []
    for c, rng in enumerate(rngs):
        n = int(rng.integers(100, 1001))
        t = _nightly_times(rng, nights, n, replace=False)
        dy = _ztf_sigma(rng, n)
        y = dy * rng.standard_normal(n)
        u = rng.random()
        if u < 0.1:
            amp = _log_uniform(rng, 0.01, 0.1)
            f0 = _log_uniform(rng, 0.1, 20.0)
            ph0 = rng.random()
            y += amp * np.sin(2.0 * np.pi * (f0 * t + ph0))
            labels.append(dict(kind="sinusoid", f0=f0, amp=amp))
        elif u < 0.2:
            depth = rng.uniform(0.1, 0.5)
            f0 = _log_uniform(rng, 0.1, 20.0)
            ph0 = rng.random()
            phase = np.mod(f0 * t + ph0, 1.0)
            y += depth * _waveform("eclipse", phase, 0.05)
            labels.append(dict(kind="eclipse", f0=f0, amp=depth, duty=0.05))
        else:
            labels.append(dict(kind="noise", f0=0.0, amp=0.0))
        curves.append((t, y, dy))
    return _assemble(curves, _grid("ztf"), BINS["ztf"], labels, "ztf_batch")


def _mixed_waveform_curve(rng, t, dy, f0):
    kind = ("sinusoid", "eclipse", "sawtooth", "double")[int(rng.integers(0, 4))]
    duty = float(rng.uniform(0.02, 0.1)) if kind == "eclipse" else 0.0
    ph0 = rng.random()
    s = _waveform(kind, np.mod(f0 * t + ph0, 1.0), duty)
    snr_target = rng.uniform(3.0, 20.0)
    snr = _signal_to_noise(s, dy)
    amp = snr_target / snr if snr > 0 else 0.0
    return amp * s, dict(kind=kind, f0=f0, amp=amp, duty=duty, snr=snr_target)


def uneven_batch(n_curves: int = 100_000) -> Batch:
    """Uneven lengths (lognormal, 50-2000), 500-2000 d baselines, four waveform kinds."""
    rngs = _seed("uneven", n_curves)
    curves, labels = [], []
    for rng in rngs:
        n = int(np.clip(np.round(np.exp(rng.normal(np.log(300.0), 0.8))), 50, 2000))
        T = rng.uniform(500.0, 2000.0)
        nights = _observable_nights(T)
        t = _nightly_times(rng, nights, n, replace=n > len(nights))
        dy = _ztf_sigma(rng, n)
        f0 = _log_uniform(rng, 0.1, 20.0)
        s, lab = _mixed_waveform_curve(rng, t, dy, f0)
        curves.append((t, s + dy * rng.standard_normal(n), dy))
        labels.append(lab)
    return _assemble(curves, _grid("uneven"), BINS["uneven"], labels, "uneven_batch")


def stress_batch(n_curves: int = 20_000) -> Batch:
    """3000 uniform times over 2000 d per curve, periods down to ~10 min, M = 50."""
    rngs = _seed("stress", n_curves)
    curves, labels = [], []
    for rng in rngs:
        n = 3000
        t = np.sort(rng.uniform(0.0, 2000.0, n))
        dy = _ztf_sigma(rng, n)
        f0 = _log_uniform(rng, 0.5, 150.0)
        s, lab = _mixed_waveform_curve(rng, t, dy, f0)
        curves.append((t, s + dy * rng.standard_normal(n), dy))
        labels.append(lab)
    return _assemble(curves, _grid("stress"), BINS["stress"], labels, "stress_batch")


def _ztf_signal(rng, t, dy):
    """80% noise, 10% sinusoids, 10% box eclipses, as in the ZTF-like batch."""
    n = len(t)
    y = dy * rng.standard_normal(n)
    u = rng.random()
    if u < 0.1:
        amp = _log_uniform(rng, 0.01, 0.1)
        f0 = _log_uniform(rng, 0.1, 20.0)
        y += amp * np.sin(2.0 * np.pi * (f0 * t + rng.random()))
        return y, dict(kind="sinusoid", f0=f0, amp=amp)
    if u < 0.2:
        depth = rng.uniform(0.1, 0.5)
        f0 = _log_uniform(rng, 0.1, 20.0)
        y += depth * _waveform("eclipse", np.mod(f0 * t + rng.random(), 1.0), 0.05)
        return y, dict(kind="eclipse", f0=f0, amp=depth, duty=0.05)
    return y, dict(kind="noise", f0=0.0, amp=0.0)


def shared_batch(n_curves: int = 1000, n_points: int = 500) -> Batch:
    """One image field: n_curves sources observed at the same n_points ZTF-like epochs over 1500 d.

    Each source has its own lognormal errors and signal (ZTF-like mix); M = 20,
    1e5 frequencies 0.05-50 /d.
    """
    rngs = _seed("shared", n_curves + 1)
    t = _nightly_times(rngs[0], _observable_nights(1500.0), n_points, replace=False)
    curves, labels = [], []
    for rng in rngs[1:]:
        dy = _ztf_sigma(rng, n_points)
        y, lab = _ztf_signal(rng, t, dy)
        curves.append((t, y, dy))
        labels.append(lab)
    return _assemble(curves, _grid("ztf"), BINS["ztf"], labels, "shared_batch")


def workload(name: str, n_curves: int | None = None) -> Batch:
    """Workload by name: single, ztf (1000 curves), uneven (1e5), stress (2e4)."""
    if name == "single":
        return single_curve()
    if name == "ztf":
        return ztf_batch(1000 if n_curves is None else n_curves)
    if name == "uneven":
        return uneven_batch(100_000 if n_curves is None else n_curves)
    if name == "stress":
        return stress_batch(20_000 if n_curves is None else n_curves)
    if name == "shared":
        return shared_batch(1000 if n_curves is None else n_curves)
    raise ValueError(name)


def random_batch(
    seed: int,
    n_curves: int,
    n_min: int,
    n_max: int,
    freqs: np.ndarray,
    n_bins: int,
    t_max: float = 1500.0,
) -> Batch:
    """Small ragged batches for parity tests: uniform times, lognormal errors, mixed signals."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2502, 243, 1000 + seed])))
    curves, labels = [], []
    for _ in range(n_curves):
        n = int(rng.integers(n_min, n_max + 1))
        t = np.sort(rng.uniform(0.0, t_max, n))
        dy = _ztf_sigma(rng, n)
        f0 = _log_uniform(rng, 0.1, 20.0)
        s, lab = _mixed_waveform_curve(rng, t, dy, f0) if n > 1 else (np.zeros(n), dict(kind="noise", f0=0.0))
        curves.append((t, s + dy * rng.standard_normal(n), dy))
        labels.append(lab)
    return _assemble(curves, np.asarray(freqs, dtype=np.float64), n_bins, labels, f"random{seed}")


def random_shared_batch(seed: int, n_curves: int, n_points: int, freqs: np.ndarray, n_bins: int,
                        t_max: float = 1500.0) -> Batch:
    """Small shared-timestamp batches for parity tests: one set of uniform times, per-curve errors and signals."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([2502, 243, 2000 + seed])))
    t = np.sort(rng.uniform(0.0, t_max, n_points))
    curves, labels = [], []
    for _ in range(n_curves):
        dy = _ztf_sigma(rng, n_points)
        f0 = _log_uniform(rng, 0.1, 20.0)
        s, lab = _mixed_waveform_curve(rng, t, dy, f0) if n_points > 1 else (np.zeros(n_points), dict(kind="noise", f0=0.0))
        curves.append((t, s + dy * rng.standard_normal(n_points), dy))
        labels.append(lab)
    return _assemble(curves, np.asarray(freqs, dtype=np.float64), n_bins, labels, f"random_shared{seed}")
