"""Learned control variate for the Monte Carlo singlet yield (host-side orchestration).

For one system and its field sweep:

1. training data: single-wavepacket yields phi_S(Omega_r, B_{r mod nB}) from rp_propagate,
   one direction per yield (sample r of Philox stream 1, disjoint from the evaluation
   stream 0), so that n training yields see n distinct directions;
2. training: the network g(Omega, B) of rp_mlp_* fitted by Adam on mean squared error of
   targets standardised per field (the fit then measures within-field fluctuations, the
   part a control variate can remove), the last 10 % of yields held out for early stopping;
   each epoch rotates every training direction set about the field axis by a fresh angle,
   a symmetry of the yield (H, P_S and the singlet commute with the total J_z);
3. beta_B = Cov(phi, g)/Var(g) per field on the held-out yields (rp_cv_beta); beta absorbs the
   per-field scale of g;
4. mu_B = mean of g over K fresh directions of stream 2 (rp_mlp_forward, rp_yield), with its
   standard error;
5. estimate: rp_yield(phi, g, mu, beta, err mu) on the evaluation samples, i.e.
   mean(phi - beta (g - mu)), unbiased because g, beta and mu do not depend on them;
   optionally combined by rp_combine with the plain mean of the training yields, which are
   independent Monte Carlo samples of the same yield (stream 1).

Every numerical step of the method runs in librp kernels (target standardisation and the
validation loss included); this module moves device buffers between calls, picks batches and
keeps the best parameters (early stopping on the validation loss, one scalar read back per
epoch).
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
        self.beta = self.mu = self.mu_err = None
        self.history = []

    # ------------------------------------------------------------------ data
    def generate(self, n, stream=STREAM_EVAL, first=0):
        """Evaluation data: (angles [n][N][2], phi [nB][n]), every direction at every field."""
        ang = rp.sample(self.s, self.seed, n, first=first, stream_id=stream)
        phi = rp.propagate(self.s, self.B[None, :], ang, n, precision=self.precision)[0]
        return ang, phi

    def generate_training(self, n_per_field, progress=None):
        """Training data with one direction per yield: direction r (stream 1) at field r % nB.
        Returns (angles [nB*n][N][2], phi [nB*n])."""
        import torch
        nB = self.nB
        ang = rp.sample(self.s, self.seed, n_per_field * nB, stream_id=STREAM_TRAIN)
        # One call: the system once per field (each copy with its own field and directions), so
        # that every training yield shares the job queue's launches.
        per_field = torch.cat([ang[b::nB].reshape(-1) for b in range(nB)])
        out = rp.propagate([self.s] * nB, self.B[:, None], per_field, n_per_field, precision=self.precision)
        phi = out[:, 0, :].t().reshape(-1).contiguous()     # row r = s * nB + b
        if progress:
            progress(nB, nB)
        return ang, phi

    def g(self, angles):
        """Network output for every (field, sample) of shared directions: float64 [nB][M]."""
        M = angles.shape[0]
        x = rp.mlp_features(angles, self.B, self.n_in)
        y = rp.mlp_forward(self.params, x, self.n_in, self.width, self.depth)
        return y.double().reshape(self.nB, M)

    # ------------------------------------------------------------------ training
    def train(self, angles, phi, epochs=200, batch=512, lr=1e-3, val_frac=0.1, patience=10, augment=True):
        """Fits g on training data from generate_training; returns the best validation MSE in
        units of the per-field variance (1 - R^2 within fields).  With ``augment`` every epoch
        sees each training direction set rotated about the field axis by a fresh random angle
        (the yield is invariant under that rotation; rp_mlp_features rot_seed)."""
        import torch
        nB = self.nB
        n_pf = phi.shape[0] // nB
        n_val = max(2, int(round(n_pf * val_frac)))
        n_tr = n_pf - n_val
        rows_tr = n_tr * nB
        # Targets standardised per field over the training rows (row r has field r % nB).
        t = rp.mlp_standardize(phi, nB, n_pf, n_tr)
        x = rp.mlp_features(angles, self.B, self.n_in, layout=2)
        x_tr, t_tr = x[:rows_tr], t[:rows_tr]
        x_va, t_va = x[rows_tr:], t[rows_tr:]
        ws = rp.mlp_workspace(self.n_in, self.width, self.depth, max(batch, x_va.shape[0]))
        best, best_p, bad = np.inf, self.params.clone(), 0
        for ep in range(epochs):
            x_ep = x_tr
            if augment:
                x_ep = rp.mlp_features(angles, self.B, self.n_in, layout=2,
                                       rot_seed=(self.seed << 20) + ep + 1)[:rows_tr]
            for i in range(0, rows_tr - batch + 1, batch):
                self.step += 1
                rp.mlp_train_step(self.params, self.m, self.v, self.step, x_ep[i:i + batch], t_tr[i:i + batch],
                                  self.n_in, self.width, self.depth, lr=lr, workspace=ws)
            val = float(rp.mlp_loss(self.params, x_va, t_va, self.n_in, self.width, self.depth, workspace=ws))
            self.history.append(val)
            if val < best:
                best, best_p, bad = val, self.params.clone(), 0
            else:
                bad += 1
                if bad >= patience:
                    break
        self.params.copy_(best_p)
        self.val_mse = best
        # beta per field from the held-out yields (independent of any later evaluation set)
        y = rp.mlp_forward(self.params, x_va, self.n_in, self.width, self.depth, workspace=ws)
        g_va = y.double().reshape(n_val, nB).t().contiguous()
        phi_va = phi[rows_tr:].reshape(n_val, nB).t().contiguous()
        self.beta = rp.cv_beta(phi_va, g_va)
        # The training yields are also plain Monte Carlo samples (stream 1, independent of the
        # evaluation stream): their per-field mean is a second unbiased estimate.
        self.train_mean, self.train_err = rp.yield_stats(phi.reshape(n_pf, nB).t().contiguous())
        return best

    def fit_mu(self, K, first=0):
        """mu_B = E[g(., B)] from K directions of the quadrature stream, and its standard error."""
        ang = rp.sample(self.s, self.seed, K, first=first, stream_id=STREAM_QUAD)
        self.mu, self.mu_err = rp.yield_stats(self.g(ang))
        return self.mu, self.mu_err

    # ------------------------------------------------------------------ estimate
    def estimate(self, angles, phi, with_training=False):
        """Control-variate mean and standard error per field for evaluation samples; with
        ``with_training`` combined (inverse-variance weights) with the plain mean of the
        training yields."""
        g = self.g(angles)
        m, e = rp.yield_stats(phi, g, self.mu, self.beta, self.mu_err)
        if with_training:
            m, e = rp.combine(m, e, self.train_mean, self.train_err)
        return m, e
