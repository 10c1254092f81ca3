"""Workload configurations for model-based iterative edge-illumination tomography.

Units (a reading of the paper, which states none for the discrete problem):
lengths in detector pixels (voxel pitch = detector pitch = 1), mask offsets m and
refraction shifts Delta in mask periods, kappa = sample-detector distance expressed
in mask periods per unit refraction angle, so that Delta = kappa * d/dt R[delta]
(the forward model of eq. 2 / eq. 4 with m_o = m_r = 0).

The mu range [0, 0.05]/px is read as normalised to a 64-voxel field of view:
at grid size N the top of the range is 0.05*64/N, so the largest projected
attenuation (about 1.5) and hence the transmission range is the same at every
grid size (0.05/px at N = 512 would give line integrals near 20, i.e. no photons).
The delta range [0, 1e-3] is kept at every N: the refraction shift follows the
slope of the delta projection, which does not grow with N.

The regularisation weight lam (eq. 5, lambda = 1e-2 as in the experiment section)
is applied to the scaled unknowns z = [mu / mu_scale ; delta / delta_scale], so in
raw units lam_mu = lam / mu_scale**2 and lam_delta = lam / delta_scale**2.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple


def mu_range_for(n: int) -> float:
    """Top of the mu range at grid size n (0.05/px normalised to 64 voxels)."""
    return 0.05 * 64.0 / n


@dataclass(frozen=True)
class SliceConfig:
    """One 2-D slice problem: grid, angles, detector, mask positions, phantom recipe."""
    n: int                      # reconstruction grid is n x n voxels
    n_theta: int                # projection angles, uniform over [0, pi)
    n_det: int                  # detector pixels
    n_mask: int                 # sample-mask positions per illumination curve
    phantom: str = "random"     # "random" ellipses or "shepp" (Shepp-Logan-style)
    n_ellipses: int = 6
    axis_max: float = 0.4       # random ellipses: semi-axes U[0.08, axis_max] * n/2
    sigma: float = 0.6          # flat IC Gaussian width, mask periods
    sigma_jitter: float = 0.0   # per-pixel relative jitter of sigma (uniform +-)
    counts: float = 1e4         # flat-field peak counts (Poisson level)
    kappa: float = 10.0
    lam: float = 1e-2
    mu_scale: float = 0.05      # top of the mu range, per pixel (see mu_range_for)
    delta_scale: float = 1e-3   # delta range [0, 1e-3]
    iters: int = 50
    seed: int = 0
    # acquisition and object variants of the full model (eq. 4); defaults = the plain model
    angle_span: float = 1.0     # angles theta_a = a * angle_span * pi / n_theta (2.0: 360 deg)
    mask_list: Tuple[float, ...] = ()   # explicit mask positions (default: spread over a period)
    gamma_h: float = 0.0        # > 0: homogeneous object, delta = gamma_h * mu
    flat_scans: int = 0         # >= 1: the flat IC is measured (tabulated, Poisson noise at
                                # flat_scans * counts photons) instead of known analytically
    n_table: int = 33           # flat IC samples over one mask period (tabulated flats)
    drift_amp: float = 0.0      # amplitude (periods) of a seeded per-angle mask drift m_o

    @property
    def lam_mu(self) -> float:
        return self.lam / self.mu_scale ** 2

    @property
    def lam_delta(self) -> float:
        return self.lam / self.delta_scale ** 2


# Plain method, CPU-sized: 64^2 grid, 90 angles over 180 deg, 64 detector pixels,
# 5 mask positions, 6 random ellipses, sigma 0.6, Poisson at 1e4, 50 iterations.
SMALL_64 = SliceConfig(n=64, n_theta=90, n_det=64, n_mask=5, phantom="random",
                       n_ellipses=6, sigma=0.6, sigma_jitter=0.0, iters=50)

# Plain method at paper-like size: 512^2, 720 angles, 512 pixels, 8 mask positions,
# per-pixel sigma jittered +-5 %, Shepp-Logan-style phantom, 100 iterations.
SLICE_512 = SliceConfig(n=512, n_theta=720, n_det=512, n_mask=8, phantom="shepp",
                        n_ellipses=10, sigma=0.6, sigma_jitter=0.05, iters=100,
                        mu_scale=0.05 * 64 / 512)

# Differentiation workload: 1024^2, 1800 angles, 1024 pixels, 12 mask positions.
SLICE_1024 = SliceConfig(n=1024, n_theta=1800, n_det=1024, n_mask=12, phantom="shepp",
                         n_ellipses=10, sigma=0.6, sigma_jitter=0.05, iters=100,
                         mu_scale=0.05 * 64 / 1024)


@dataclass(frozen=True)
class BatchConfig:
    """Many independent slices of mixed size in one launch (3-D = stack of 2-D)."""
    n_slices: int = 256
    classes: Tuple[Tuple[int, int], ...] = ((256, 360), (512, 720), (768, 1080))
    n_mask: int = 8
    n_ellipses: int = 6
    sigma: float = 0.6
    sigma_jitter: float = 0.05
    iters: int = 100
    seed: int = 0

    def slice_configs(self):
        """Seeded shuffle of size classes (85/85/86 split for 256 slices)."""
        import numpy as np
        k = len(self.classes)
        counts = [self.n_slices // k] * k
        for i in range(self.n_slices - sum(counts)):
            counts[k - 1 - i] += 1
        labels = np.concatenate([np.full(c, i) for i, c in enumerate(counts)])
        rng = np.random.default_rng(self.seed)
        rng.shuffle(labels)
        out = []
        for s, lab in enumerate(labels):
            n, nt = self.classes[int(lab)]
            out.append(SliceConfig(n=n, n_theta=nt, n_det=n, n_mask=self.n_mask,
                                   phantom="random", n_ellipses=self.n_ellipses,
                                   sigma=self.sigma, sigma_jitter=self.sigma_jitter,
                                   iters=self.iters, seed=s,
                                   mu_scale=mu_range_for(n)))
        return out


BATCH_256 = BatchConfig()


@dataclass(frozen=True)
class WarmStartConfig:
    """Learned warm start: 4-level U-Net, 32 base channels, trained at 256^2/360 on 4000
    random-ellipse slices, evaluated at 512^2/720."""
    train_n: int = 256
    train_theta: int = 360
    n_mask: int = 8
    n_train: int = 4000
    n_val: int = 128
    epochs: int = 80
    target_iters: int = 300
    eval_n: int = 512
    eval_theta: int = 720
    n_eval: int = 32
    eval_seed0: int = 1_000_000
    base_channels: int = 32
    levels: int = 4
    tol: float = 1e-3


WARMSTART = WarmStartConfig()

# The paper's own acquisition (experiment section): homogeneous object (mu = h, delta = gamma h,
# gamma = 5), one mask position on the slope of the IC, 400 projections over 360 degrees, a
# 220^2 grid, lambda = 1e-2. The IC is narrower than the plain workloads' (sigma 0.3 period,
# the position m = 0.3 on its steepest slope) and kappa = 0.3, so that the refraction shifts
# of the granule-like phantom stay near 0.1 period (with kappa = 1 they reach a period at
# object edges, where the central-difference model cannot follow the data); the flat IC is
# measured over one period in 33 steps (1 or 20 flat scans) and the mask drifts by up to
# 0.02 period.
PAPER_220 = SliceConfig(n=220, n_theta=400, n_det=220, n_mask=1, phantom="random",
                        n_ellipses=12, axis_max=0.3, sigma=0.3, sigma_jitter=0.05, kappa=0.3,
                        iters=100, mu_scale=0.05 * 64 / 220, angle_span=2.0, mask_list=(0.3,),
                        gamma_h=5.0, flat_scans=20, n_table=33, drift_amp=0.02)

CONFIGS = {"small_64": SMALL_64, "slice_512": SLICE_512, "slice_1024": SLICE_1024,
           "paper_220": PAPER_220}


def with_seed(cfg: SliceConfig, seed: int) -> SliceConfig:
    return replace(cfg, seed=seed)
