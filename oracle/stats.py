"""Monte Carlo statistics of the trace estimate (Eq. 18, Eq. 23).  Test infrastructure only."""
import numpy as np


def mc_mean_error(phi):
    """Mean over samples and its standard error eps = s / sqrt(M) (Eq. 23).

    ``phi`` is [..., M]; s uses the unbiased 1/(M-1) normalisation (sigma is
    estimated from the M samples, as in the caption of Fig. 2).
    """
    phi = np.asarray(phi, float)
    M = phi.shape[-1]
    mean = phi.mean(axis=-1)
    if M < 2:
        return mean, np.zeros_like(mean)
    s = phi.std(axis=-1, ddof=1)
    return mean, s / np.sqrt(M)


def cv_mean_error(phi, g, mu, beta, mu_err=None):
    """Control-variate estimate mean(phi - beta (g - mu)) and its standard error.

    With beta and mu fixed independently of the evaluation samples the
    estimator is unbiased for E[phi]; its error is s'/sqrt(M) with s' the
    sample deviation of phi - beta g.
    """
    phi = np.asarray(phi, float)
    g = np.asarray(g, float)
    mu = np.asarray(mu, float)[..., None]
    beta = np.asarray(beta, float)[..., None]
    m, e = mc_mean_error(phi - beta * (g - mu))
    if mu_err is not None:
        e = np.sqrt(e * e + (beta[..., 0] * np.asarray(mu_err, float)) ** 2)
    return m, e


def combine(mean_a, err_a, mean_b, err_b):
    """Inverse-variance weighted mean of two independent unbiased estimates and its error:
    the minimum-variance unbiased linear combination for fixed weights."""
    ma, ea, mb, eb = (np.asarray(x, float) for x in (mean_a, err_a, mean_b, err_b))
    va, vb = ea * ea, eb * eb
    with np.errstate(divide="ignore", invalid="ignore"):
        m = np.where(va == 0, ma, np.where(vb == 0, mb, (ma / va + mb / vb) / (1 / va + 1 / vb)))
        e = np.where((va == 0) | (vb == 0), 0.0, 1 / np.sqrt(1 / va + 1 / vb))
    return m, e
