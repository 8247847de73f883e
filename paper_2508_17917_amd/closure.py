"""Learned closure: a per-element network that corrects an order-lo solution
toward the order-hi one on the same mesh (binding of the dg_mlp_* and
dg_closure_* calls; every array operation runs in the library's kernels).

Samples come from order-hi states (restricted to order lo); the network is
trained on them with Adam on the GPU; a corrected state is I U_lo + y.  The
order-hi solve stays the reference: `needs_fallback` flags states whose
samples leave the range the network was trained on (any input column whose
mean moves by more than `tol` training standard deviations, or whose spread
grows beyond `tol` times the training one), where the caller should run
the order-hi solver instead.
"""
import numpy as np

from . import _lib as L


class Closure:
    def __init__(self, lo, hi, n_hidden=128, max_batch=1 << 16, params=None):
        """lo, hi: set-up Solvers of orders lo < hi on the same mesh."""
        import torch
        self.lo, self.hi = lo, hi
        self.c = L.dg_closure_create(lo.h, hi.h)
        self.n_in, self.n_out = L.dg_closure_sizes(self.c)
        self.m = L.dg_mlp_create(self.n_in, n_hidden, self.n_out, max_batch)
        self.n_hidden = n_hidden
        self.max_batch = max_batch
        self.K = hi.K
        if params is not None:
            L.dg_mlp_set_params(self.m, params)
        self.in_stats = None
        self._torch = torch

    def rebind(self, lo, hi):
        """Use the trained network with another pair of solvers (same orders;
        e.g. other physics on the same or another mesh)."""
        c = L.dg_closure_create(lo.h, hi.h)
        if L.dg_closure_sizes(c) != (self.n_in, self.n_out):
            L.dg_closure_destroy(c)
            raise ValueError("the new solvers have other orders")
        L.dg_closure_destroy(self.c)
        self.c, self.lo, self.hi, self.K = c, lo, hi, hi.K

    # -- samples
    def features(self, U, from_hi, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty((self.K, self.n_in), dtype=torch.float32, device="cuda")
        L.dg_closure_features(self.c, U, out, from_hi)
        return out

    def targets(self, U_hi, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty((self.K, self.n_out), dtype=torch.float32, device="cuda")
        L.dg_closure_targets(self.c, U_hi, out)
        return out

    def samples(self, U_hi):
        return self.features(U_hi, True), self.targets(U_hi)

    # -- network
    def set_params(self, params):
        L.dg_mlp_set_params(self.m, params)

    def params(self):
        return L.dg_mlp_get_params(self.m)

    def fit_normalization(self, X, T):
        """Per-column mean and standard deviation of a sample set (device
        arrays); columns that do not vary keep unit scale."""
        xm, xs = L.dg_column_stats(X, cols=self.n_in)
        tm, ts = L.dg_column_stats(T, cols=self.n_out)
        xs = np.where(xs > 1e-12 * np.maximum(1.0, np.abs(xm)), xs, 1.0)
        ts = np.where(ts > 0.0, ts, 1.0)
        L.dg_mlp_set_normalization(self.m, xm, xs, tm, ts)
        self.in_stats = (xm, xs)
        return xm, xs, tm, ts

    def predict(self, X, out=None):
        torch = self._torch
        B = X.shape[0]
        if out is None:
            out = torch.empty((B, self.n_out), dtype=torch.float32, device="cuda")
        for b0 in range(0, B, self.max_batch):
            b1 = min(B, b0 + self.max_batch)
            L.dg_mlp_forward(self.m, X[b0:b1], out[b0:b1])
        return out

    def train(self, X, T, epochs=1, batch=8192, lr=1e-3, seed=0, log=None, loss_every=1):
        """Minibatch Adam over the sample set (X, T: device arrays of equal
        length, rows in any order).  Minibatches are contiguous row ranges,
        visited in a seeded random order each epoch.  Returns the losses read
        back every `loss_every` steps (each read synchronises the stream)."""
        n = X.shape[0]
        batch = min(batch, self.max_batch, n)
        starts = np.arange(0, n - batch + 1, batch)
        rng = np.random.default_rng(seed)
        losses = []
        step = 0
        for ep in range(epochs):
            for b0 in rng.permutation(starts):
                want = (step % loss_every) == 0
                loss = L.dg_mlp_backward(self.m, X[b0:b0 + batch], T[b0:b0 + batch],
                                         want_loss=want)
                L.dg_mlp_adam(self.m, lr)
                if want:
                    losses.append(loss)
                step += 1
            if log:
                log("epoch %d: loss %.4e" % (ep, losses[-1] if losses else float("nan")))
        return losses

    # -- use
    def correct(self, U_lo, out=None):
        """Order-hi state I U_lo + network(samples of U_lo)."""
        X = self.features(U_lo, False)
        Y = self.predict(X)
        if out is None:
            out = self.hi.empty_state()
        L.dg_closure_apply(self.c, U_lo, Y, out)
        return out

    def restrict(self, U_hi, out=None):
        if out is None:
            out = self.lo.empty_state()
        L.dg_closure_restrict(self.c, U_hi, out)
        return out

    def interpolate(self, U_lo, out=None):
        if out is None:
            out = self.hi.empty_state()
        L.dg_closure_apply(self.c, U_lo, None, out)
        return out

    def correct_or_fallback(self, U_lo, reference, tol=4.0, out=None):
        """The corrected order-hi state, or reference() (the caller's order-hi
        solve) when the samples of U_lo leave the training distribution.
        Returns (state, used_fallback)."""
        if self.needs_fallback(U_lo, tol):
            return reference(), True
        return self.correct(U_lo, out), False

    def needs_fallback(self, U_lo, tol=4.0):
        if self.in_stats is None:
            return True
        X = self.features(U_lo, False)
        m, s = L.dg_column_stats(X, cols=self.n_in)
        xm, xs = self.in_stats
        return bool(np.any(np.abs(m - xm) > tol * xs) or np.any(s > tol * np.maximum(xs, 1e-300)))

    def close(self):
        if self.m is not None:
            L.dg_mlp_destroy(self.m)
            self.m = None
        if self.c is not None:
            L.dg_closure_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
