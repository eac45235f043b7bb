"""Host-side pieces of the training: the loss of Eq. (loss) and the unroll
curriculum of Sec. "Learning Task" (CPU)."""
import numpy as np

from paper_2412_08229_amd.training import curriculum_steps, n_bins, paper_spectrum_loss


def test_paper_loss_value_and_gradient():
    rng = np.random.Generator(np.random.PCG64(3))
    n = 32
    E = rng.random(n_bins(n)) * 1e-3
    Et = rng.random(n_bins(n)) * 1e-3
    L, dE = paper_spectrum_loss(E, Et, kappa_max=n // 2)
    ks = np.arange(4, 11)
    assert np.isclose(L, np.mean((E[ks] - Et[ks]) ** 2) + 20.0 * E[16], rtol=1e-14)
    # Central differences (the loss is quadratic plus linear: exact to rounding).
    h = 1e-7
    for k in list(range(len(E))):
        e = np.zeros_like(E)
        e[k] = h
        fd = (paper_spectrum_loss(E + e, Et, kappa_max=16)[0] - paper_spectrum_loss(E - e, Et, kappa_max=16)[0]) / (2 * h)
        assert abs(fd - dE[k]) < 1e-7 * max(1.0, abs(dE[k]))
    # Only the window and the cutoff shell carry gradient.
    nz = set(np.nonzero(dE)[0])
    assert nz <= set(ks) | {16} and 16 in nz
    # The default cutoff shell is N/2 for these sizes.
    for m in (16, 32, 64, 128):
        assert paper_spectrum_loss(np.ones(n_bins(m)), np.ones(n_bins(m)), omega=1.0)[0] == 1.0


def test_curriculum_schedule():
    assert [curriculum_steps(e) for e in (0, 9, 10, 19, 20, 89)] == [200, 200, 400, 400, 600, 1800]


def test_train_batched_applies_the_schedule_and_skips_failed_samples():
    """train_batched sets every sample's unroll length from the schedule
    before each epoch, averages the gradients of the samples that returned a
    finite loss, and steps Adam on them (CPU, stand-in samples whose loss is
    a quadratic in the parameters)."""
    from paper_2412_08229_amd.training import train_batched

    class Quadratic:
        def __init__(self, centre, fail_at=None):
            self.centre, self.fail_at, self.nsteps, self.seen = np.asarray(centre, float), fail_at, 0, []

        def loss_and_grad(self, p):
            self.seen.append(self.nsteps)
            if self.fail_at is not None and self.nsteps == self.fail_at:
                return float("nan"), np.zeros_like(p), None
            d = p - self.centre
            return float(d @ d), 2.0 * d, None

    runs = [Quadratic([1.0, -1.0]), Quadratic([3.0, 1.0], fail_at=40)]
    p, hist = train_batched(runs, np.zeros(2), 6, lr=0.5,
                            schedule=lambda ep: curriculum_steps(ep, start=20, grow=20, every=2))
    assert runs[0].seen == [20, 20, 40, 40, 60, 60] and runs[1].seen == runs[0].seen
    assert len(hist) == 6 and all(np.isfinite(hist))
    # Adam moves towards the mean of the centres, (2, 0).
    assert np.linalg.norm(p - np.array([2.0, 0.0])) < np.linalg.norm(np.array([2.0, 0.0]))


def test_adam_steps_do_not_depend_on_the_loss_scale():
    """Adam's epsilon is a fraction of the first gradient's RMS, so scaling
    the loss by 1e-12 (a lattice-unit spectrum loss) takes the same steps as
    the unscaled loss; with torch's fixed epsilon of 1e-8 the scaled run
    would barely move (CPU, a quadratic stand-in sample)."""
    from paper_2412_08229_amd.training import train_batched

    class Scaled:
        def __init__(self, scale):
            self.scale, self.nsteps = scale, 0

        def loss_and_grad(self, p):
            d = p - np.array([1.0, -2.0, 0.5])
            return float(self.scale * (d @ d)), self.scale * 2.0 * d, None

    p1, h1 = train_batched([Scaled(1.0)], np.zeros(3), 8, lr=0.1)
    p2, h2 = train_batched([Scaled(1e-12)], np.zeros(3), 8, lr=0.1)
    np.testing.assert_allclose(p2, p1, rtol=1e-6)
    np.testing.assert_allclose(np.array(h2) * 1e12, h1, rtol=1e-5)
    assert np.linalg.norm(p2) > 0.5                # moved ~lr per step, not lr * g / 1e-8
