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
