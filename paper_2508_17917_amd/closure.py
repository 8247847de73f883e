"""Learned closure: per-element networks that bring an order-lo solution on a
mesh toward the order-hi one (binding of the dg_mlp_* and dg_closure_*
calls; every array operation runs in the library's kernels).

Two networks on the same samples x = [Pi_lo(U - U_inf), rx, ry, sx, sy]:

* the corrector, which corrects the order-lo solve itself: every m steps of
  the order-lo solver, U_lo += net_c(x(U_lo)) - net_c(x0), trained on the
  drift of m order-lo steps from the restriction of an order-hi state,
  Pi_lo U_hi(t + m dt) - Phi_lo^m(Pi_lo U_hi(t));
* the reconstruction, which adds the part of the order-hi state that order
  lo cannot represent: I U_lo + net_r(x(U_lo)) - net_r(x0), trained on
  U_hi - I Pi_lo U_hi (Pi_lo of that part is zero, so on its own it cannot
  change the order-lo solve).

x0 is the free stream's sample of each element (its state columns zero):
both solvers leave a free-stream element unchanged and its unresolved part
is zero, so subtracting the network's output there makes both corrections
vanish exactly on undisturbed elements, where a network otherwise adds its
small residual error over the largest elements of the mesh.  Training sets
carry free-stream rows with zero targets (`free_rows`) so that the
subtracted value is itself small.

Samples come from order-hi states; the networks are trained with Adam on
the GPU.  The order-hi solve stays the reference: `needs_fallback` flags
states whose samples leave the range the networks were trained on (any
input column whose mean moves by more than `tol` training standard
deviations, or whose spread grows beyond `tol` times the training one),
where the caller should run the order-hi solver instead.
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
        self.mc = None
        self.n_lo = self.n_in - 4
        self._y0 = {}
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
        self._y0 = {}

    # -- samples
    def features(self, U, from_hi, out=None):
        """Samples of every element: from_hi 1 an order-hi state, 0 an
        order-lo state, 2 the free stream (U ignored)."""
        torch = self._torch
        if out is None:
            out = torch.empty((self.K, self.n_in), dtype=torch.float32, device="cuda")
        L.dg_closure_features(self.c, U, out, int(from_hi))
        return out

    def free_rows(self, n_out, reps=1):
        """Training rows of the free stream on this mesh: reps copies of every
        element's free-stream sample, with zero targets of width n_out."""
        torch = self._torch
        X0 = self.features(None, 2)
        X = X0.repeat(reps, 1)
        return X, torch.zeros((X.shape[0], n_out), dtype=torch.float32, device="cuda")

    def _free_output(self, net, n_out):
        """The network's output for the free-stream samples (cached per mesh
        binding and parameters)."""
        key = (id(net), n_out)
        if key not in self._y0:
            self._y0[key] = self._predict(net, self.features(None, 2), n_out)
        return self._y0[key]

    def targets(self, U_hi, out=None):
        torch = self._torch
        if out is None:
            out = torch.empty((self.K, self.n_out), dtype=torch.float32, device="cuda")
        L.dg_closure_targets(self.c, U_hi, out)
        return out

    def samples(self, U_hi):
        return self.features(U_hi, True), self.targets(U_hi)

    # -- corrector of the order-lo solve
    def make_corrector(self, params=None, n_hidden=128):
        """The corrector network (n_features -> n_hidden -> n_hidden -> 4 Np_lo)."""
        self.n_lo = self.n_in - 4
        self._y0 = {}
        if getattr(self, "mc", None) is not None:
            L.dg_mlp_destroy(self.mc)
        self.mc = L.dg_mlp_create(self.n_in, n_hidden, self.n_lo, self.max_batch)
        if params is not None:
            L.dg_mlp_set_params(self.mc, params)
        return self.mc

    def drift_rows(self, U_lo, U_hi_later, X=None, T=None):
        """Corrector samples from an order-lo state after m steps from the
        restriction of an order-hi state, and that order-hi state m steps
        later: x = sample of U_lo, t = Pi_lo U_hi_later - U_lo."""
        torch = self._torch
        if X is None:
            X = torch.empty((self.K, self.n_in), dtype=torch.float32, device="cuda")
        if T is None:
            T = torch.empty((self.K, self.n_lo), dtype=torch.float32, device="cuda")
        self.features(U_lo, False, out=X)
        L.dg_closure_drift_targets(self.c, self.restrict(U_hi_later), U_lo, T)
        return X, T

    def correct_lo(self, U_lo):
        """U_lo += corrector(samples of U_lo) - corrector(free stream), in place."""
        X = self.features(U_lo, False)
        Y = self._predict(self.mc, X, self.n_lo)
        L.dg_closure_correct(self.c, Y, U_lo, Y0=self._free_output(self.mc, self.n_lo))
        return U_lo

    def corrected_steps(self, U_lo, K1, nsteps, dt, m, v_w=(0.0, 0.0), phase=0):
        """nsteps order-lo LSERK steps with the corrector applied after every
        step whose count (from phase) is a multiple of m.  Returns the new
        phase (steps since the last correction)."""
        done = 0
        while done < nsteps:
            n = min(m - phase, nsteps - done)
            self.lo.rk_steps(U_lo, K1, n, dt, v_w)
            done += n
            phase += n
            if phase == m:
                self.correct_lo(U_lo)
                phase = 0
        return phase

    def fit_corrector_normalization(self, X, T):
        return self._fit(self.mc, X, T, self.n_lo, corrector=True)

    def train_corrector(self, X, T, **kw):
        return self._train(self.mc, X, T, **kw)

    # -- reconstruction network
    def set_params(self, params):
        L.dg_mlp_set_params(self.m, params)
        self._y0 = {}

    def params(self):
        return L.dg_mlp_get_params(self.m)

    def _fit(self, net, X, T, n_out, corrector=False):
        self._y0 = {}
        xm, xs = L.dg_column_stats(X, cols=self.n_in)
        tm, ts = L.dg_column_stats(T, cols=n_out)
        xs = np.where(xs > 1e-12 * np.maximum(1.0, np.abs(xm)), xs, 1.0)
        ts = np.where(ts > 0.0, ts, 1.0)
        L.dg_mlp_set_normalization(net, xm, xs, tm, ts)
        if not corrector or self.in_stats is None:
            self.in_stats = (xm, xs)
        return xm, xs, tm, ts

    def fit_normalization(self, X, T):
        """Per-column mean and standard deviation of a sample set (device
        arrays); columns that do not vary keep unit scale."""
        return self._fit(self.m, X, T, self.n_out)

    def _predict(self, net, X, n_out, out=None):
        torch = self._torch
        B = X.shape[0]
        if out is None:
            out = torch.empty((B, n_out), dtype=torch.float32, device="cuda")
        for b0 in range(0, B, self.max_batch):
            b1 = min(B, b0 + self.max_batch)
            L.dg_mlp_forward(net, X[b0:b1], out[b0:b1])
        return out

    def predict(self, X, out=None):
        return self._predict(self.m, X, self.n_out, out)

    def _train(self, net, X, T, epochs=1, batch=8192, lr=1e-3, seed=0, log=None, loss_every=1):
        self._y0 = {}
        n = X.shape[0]
        batch = min(batch, self.max_batch, n)
        starts = np.arange(0, n - batch + 1, batch)
        rng = np.random.default_rng(seed)
        losses = []
        step = 0
        for ep in range(epochs):
            for b0 in rng.permutation(starts):
                want = (step % loss_every) == 0
                loss = L.dg_mlp_backward(net, X[b0:b0 + batch], T[b0:b0 + batch], want_loss=want)
                L.dg_mlp_adam(net, lr)
                if want:
                    losses.append(loss)
                step += 1
            if log:
                log("epoch %d: loss %.4e" % (ep, losses[-1] if losses else float("nan")))
        return losses

    def train(self, X, T, **kw):
        """Minibatch Adam over the sample set (X, T: device arrays of equal
        length, rows in any order).  Minibatches are contiguous row ranges,
        visited in a seeded random order each epoch.  Returns the losses read
        back every `loss_every` steps (each read synchronises the stream)."""
        return self._train(self.m, X, T, **kw)

    # -- use
    def correct(self, U_lo, out=None):
        """Order-hi state I U_lo + network(samples of U_lo) - network(free stream)."""
        X = self.features(U_lo, False)
        Y = self.predict(X)
        if out is None:
            out = self.hi.empty_state()
        L.dg_closure_apply(self.c, U_lo, Y, out, Y0=self._free_output(self.m, self.n_out))
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
        if getattr(self, "mc", None) is not None:
            L.dg_mlp_destroy(self.mc)
            self.mc = None
        if self.c is not None:
            L.dg_closure_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
