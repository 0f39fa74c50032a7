"""Lucy-Richardson initialisation of FSMP (Sec. 2.3), plain numpy in FP64.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline leg of
the benchmark; the product library neither loads nor calls it, and it shares no code with
the HIP path.

What it computes, per waveform w of L_w samples (1 ns apart) and the single-PE response
V sampled at whole samples s = 0 .. L_V - 1:

* the iterative deconvolution of Lucy (1974) in the two-sum form of Sec. 2.3, over
  tau in [-L_V + 1, L_w - 1] and t in [0, L_w - 1]:
      w^r(t)        = sum over tau in [t - L_V + 1, t] of qhat^r(tau) K(t - tau)
      qhat^{r+1}(tau) = qhat^r(tau) sum over t in [max(tau, 0), min(L_w - 1, tau + L_V - 1)]
                        of d(t) / w^r(t) K(t - tau)
  (the limits of the first sum as printed in the paper give an empty range; these are the
  limits of the convolution they describe);
* the initial PE sequence {tau : qhat(tau) > threshold}, the solution space
  T = [t_min - margin, t_max + margin] and the waveform cut
  [t_min - margin, t_max + margin + L_V] (Sec. 2.3, solution space), and the first PE
  time as the initial t0.

Readings where the paper leaves a choice (each is listed in the design notes):
* K = V / sum_s V(s), the response normalised to unit sum: the multiplicative update has
  the data as its fixed point only then, and qhat = (deconvolved flux) / sum_s V(s) is in
  units of one PE's charge, the unit of the 0.1 threshold;
* d = max(w, 0): the update needs non-negative data; a ratio with w^r(t) = 0 counts 0;
* qhat^0 uniform over the L_w + L_V - 1 points with total sum(d) (any non-negative start
  with the data's total is allowed);
* only tau >= 0 become PEs (the model has no PE before the window); when more than kmax
  points pass the threshold the kmax largest qhat are kept (ties: earlier tau), listed in
  time order; PE tau sits on grid index sub * tau;
* t0_init = the first PE time minus half a grid step (phi is positive at every PE), held
  inside the t0 prior; PEs at or before t0_init (only possible when the prior clamps it)
  are dropped; an empty list gives an empty T (the waveform is taken as no PE) and the
  middle of the prior as t0;
* the initial intensity scale is the total of qhat.
"""
import numpy as np


def ser_samples(p, LV):
    """V(s) at whole samples s = 0 .. LV - 1 from the oracle's SER table V(m / sub)."""
    from . import ser_table
    tab, _ = ser_table(p)
    v = np.zeros(LV)
    m = np.arange(LV) * p.sub
    ok = m < len(tab)
    v[ok] = tab[m[ok]]
    return v


def lucy(w, V, n_iter):
    """qhat after n_iter iterations, over tau = -L_V + 1 .. L_w - 1, in PE-charge units."""
    w = np.asarray(w, np.float64)
    V = np.asarray(V, np.float64)
    Lw, LV = len(w), len(V)
    A = V.sum()
    K = V / A
    d = np.maximum(w, 0.0)
    n_tau = Lw + LV - 1
    u = np.full(n_tau, d.sum() / n_tau)       # index i <-> tau = i - (LV - 1)
    for _ in range(n_iter):
        # w^r(t): the full convolution of qhat with K, at t + L_V - 1
        wr = np.convolve(u, K)[LV - 1:LV - 1 + Lw]
        ratio = np.where(wr > 0, d / np.where(wr > 0, wr, 1.0), 0.0)
        # sum over t of ratio(t) K(t - tau): a correlation of the zero-padded ratio with K
        rp = np.concatenate([np.zeros(LV - 1), ratio, np.zeros(LV - 1)])
        u = u * np.correlate(rp, K, "valid")
    return u / A


def initial_state(qhat, LV, sub, threshold, margin, kmax, t0_min, t0_max, Lw):
    """Initial PE grid list, T = [g_lo, g_hi], t0, intensity scale and the sample cut."""
    qhat = np.asarray(qhat, np.float64)
    taus = np.arange(len(qhat)) - (LV - 1)
    sel = np.nonzero((qhat > threshold) & (taus >= 0))[0]
    if len(sel) > kmax:
        order = sorted(sel, key=lambda i: (-qhat[i], i))
        sel = np.sort(np.array(order[:kmax]))
    lam = float(qhat.sum())
    if len(sel) == 0:
        return {"z": [], "g_range": (1, 0), "t0": 0.5 * (t0_min + t0_max), "lam": lam, "cut": (0, Lw - 1)}
    t_min, t_max = int(taus[sel[0]]), int(taus[sel[-1]])
    t0 = min(max(t_min - 0.5 / sub, t0_min), t0_max)
    z = [int(sub * taus[i]) for i in sel if taus[i] - t0 > 0]
    g_lo = max(0, sub * (t_min - margin))
    g_hi = min(sub * Lw - 1, sub * (t_max + margin))
    cut = (max(0, t_min - margin), min(Lw - 1, t_max + margin + LV))
    return {"z": z, "g_range": (g_lo, g_hi), "t0": t0, "lam": lam, "cut": cut}
