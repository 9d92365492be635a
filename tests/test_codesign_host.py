"""Host logic of the co-design loop (Sec. 3.2): the convergence rule and the
projection-sharpness schedule."""
from paper_2503_22767_amd import codesign as CD


def test_convergence_needs_two_full_windows():
    assert not CD.converged([1.0] * 19)
    assert CD.converged([1.0] * 20)


def test_convergence_compares_window_means():
    # means 1.0 and 1.0005: relative change 5e-4 < 1e-3
    assert CD.converged([1.0] * 10 + [1.0005] * 10)
    # means 1.0 and 1.002: 2e-3
    assert not CD.converged([1.0] * 10 + [1.002] * 10)
    # only the last 20 values count
    assert CD.converged([50.0] * 7 + [-2.0] * 10 + [-2.001] * 10)


def test_beta_doubles_every_ten_iterations_up_to_128():
    assert [CD.beta_at(i) for i in (0, 9, 10, 19, 20, 69, 70, 200)] == [1, 1, 2, 2, 4, 64, 128, 128]
    assert CD.beta_at(35, beta0=2.0, factor=4.0, every=5, beta_max=1000) == 1000
