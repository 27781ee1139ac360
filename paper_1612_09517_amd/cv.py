"""Learned control variate for the Monte Carlo singlet yield (host-side orchestration).

For one system and its field sweep:

1. training data: single-wavepacket yields phi_S(Omega, B) from rp_propagate on samples of
   Philox stream 1 (disjoint from the evaluation stream 0);
2. training: the network g(Omega, B) of rp_mlp_* fitted by Adam on mean squared error of
   standardised targets, with the last 10 % of samples held out for early stopping;
3. beta_B = Cov(phi, g)/Var(g) per field on the held-out samples (rp_cv_beta);
4. mu_B = mean of g over K fresh directions of stream 2 (rp_mlp_forward, rp_yield), with its
   standard error;
5. estimate: rp_yield(phi, g, mu, beta, err mu) on the evaluation samples, i.e.
   mean(phi - beta (g - mu)), unbiased because g, beta and mu do not depend on them.

Every numerical step runs in librp kernels; this module only moves device buffers between
calls, picks batches and keeps the best parameters (early stopping on a host-side scalar).
"""
import numpy as np

from . import rp

STREAM_EVAL, STREAM_TRAIN, STREAM_QUAD = 0, 1, 2


class ControlVariate:
    def __init__(self, system, fields_mT, seed, width=256, depth=3, precision=32, init_seed=0):
        import torch
        self.s = system
        self.B = np.asarray(fields_mT, np.float64).reshape(-1)
        self.nB = len(self.B)
        self.seed = seed
        self.width, self.depth = width, depth
        self.precision = precision
        self.n_in = 3 * system.N + 1
        self.n_pad = rp.mlp_in_pad(self.n_in)
        rng = np.random.default_rng(init_seed)
        p = []
        fan = self.n_pad
        for _ in range(depth):           # He initialisation of the packed parameters
            p.append(rng.normal(0.0, np.sqrt(2.0 / fan), fan * width))
            p.append(np.zeros(width))
            fan = width
        p.append(rng.normal(0.0, np.sqrt(1.0 / width), width))
        p.append(np.zeros(1))
        host = np.concatenate(p).astype(np.float32)
        assert len(host) == rp.mlp_param_count(self.n_in, width, depth)
        self.params = torch.tensor(host, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.t_mean, self.t_std = 0.0, 1.0
        self.beta = self.mu = self.mu_err = None
        self.history = []

    # ------------------------------------------------------------------ data
    def generate(self, n, stream=STREAM_TRAIN, first=0):
        """(angles [n][N][2], phi [nB][n]) from the method itself."""
        ang = rp.sample(self.s, self.seed, n, first=first, stream_id=stream)
        phi = rp.propagate(self.s, self.B[None, :], ang, n, precision=self.precision)[0]
        return ang, phi

    def g(self, angles):
        """Network output for every (field, sample): float64 [nB][M]."""
        M = angles.shape[0]
        x = rp.mlp_features(angles, self.B, self.n_in)
        y = rp.mlp_forward(self.params, x, self.n_in, self.width, self.depth)
        return y.double().reshape(self.nB, M)

    # ------------------------------------------------------------------ training
    def train(self, angles, phi, epochs=60, batch=512, lr=1e-3, val_frac=0.1, patience=10):
        import torch
        n = angles.shape[0]
        n_val = max(1, int(round(n * val_frac)))
        n_tr = n - n_val
        # Targets: the yields, standardised on the host (input preparation), row s*nB + b.
        ph_h = phi.detach().cpu().numpy()
        self.t_mean = float(ph_h[:, :n_tr].mean())
        self.t_std = float(ph_h[:, :n_tr].std()) or 1.0
        t = torch.tensor(((ph_h.T.reshape(-1) - self.t_mean) / self.t_std).astype(np.float32), device="cuda")
        x = rp.mlp_features(angles, self.B, self.n_in, sample_major=True)
        rows_tr = n_tr * self.nB
        x_tr, t_tr = x[:rows_tr], t[:rows_tr]
        x_va, t_va = x[rows_tr:], t[rows_tr:]
        ws = rp.mlp_workspace(self.n_in, self.width, self.depth, max(batch, x_va.shape[0]))
        best, best_p, bad = np.inf, self.params.clone(), 0
        t_va_h = t_va.cpu().numpy()
        for ep in range(epochs):
            for i in range(0, rows_tr - batch + 1, batch):
                self.step += 1
                rp.mlp_train_step(self.params, self.m, self.v, self.step, x_tr[i:i + batch], t_tr[i:i + batch],
                                  self.n_in, self.width, self.depth, lr=lr, workspace=ws)
            y = rp.mlp_forward(self.params, x_va, self.n_in, self.width, self.depth, workspace=ws)
            val = float(np.mean((y.cpu().numpy() - t_va_h) ** 2))
            self.history.append(val)
            if val < best:
                best, best_p, bad = val, self.params.clone(), 0
            else:
                bad += 1
                if bad >= patience:
                    break
        # Keep the best parameters and fold the target scaling into the output layer, so that
        # g is on the scale of phi_S.
        p = best_p.cpu().numpy().astype(np.float64)
        p[-self.width - 1:-1] *= self.t_std
        p[-1] = p[-1] * self.t_std + self.t_mean
        self.params.copy_(torch.tensor(p.astype(np.float32), device="cuda"))
        self.val_mse = best            # in units of the target variance: 1 - R^2 over all fields
        # beta from the held-out samples (independent of any later evaluation set)
        g_va = self.g(angles[n_tr:])
        self.beta = rp.cv_beta(phi[:, n_tr:].contiguous(), g_va)
        return best

    def fit_mu(self, K, first=0):
        """mu_B = E[g(., B)] from K directions of the quadrature stream, and var(mu_B)."""
        ang = rp.sample(self.s, self.seed, K, first=first, stream_id=STREAM_QUAD)
        gq = self.g(ang)
        self.mu, self.mu_err = rp.yield_stats(gq)
        return self.mu, self.mu_err

    # ------------------------------------------------------------------ estimate
    def estimate(self, angles, phi):
        """Control-variate mean and standard error per field for evaluation samples."""
        g = self.g(angles)
        return rp.yield_stats(phi, g, self.mu, self.beta, self.mu_err)
