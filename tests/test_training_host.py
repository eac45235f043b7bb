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
