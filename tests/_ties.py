"""Near-tie detection for comparing the device lambda searches with the oracle's.

Both sides evaluate the same trials in FP64, but the device sums in another order, so a residual can
differ in its last digits. A search decision (accept or reject, the order of simplex vertices, the
convergence test rho <= eps) can then flip only where the two values it compares are that close.
A point whose device trajectory differs from the oracle's is acceptable only if the oracle's own
trajectory holds such a near-tie: two finite values of Phi within TIE_REL of each other, or a rho
within TIE_REL of eps.

TIE_REL = 1e-9: the FP64 device field agrees with the oracle to ~1e-14 relative; f = |J x B|/(|J||B|)
loses up to a factor 1/f of that to cancellation, so Phi and rho carry at most ~1e-10 relative error
for f >= 1e-4, the smallest residual the searches here aim at.
"""
import numpy as np

TIE_REL = 1e-9


class Recording:
    """Wraps an oracle per-point problem and records (Phi, rho) of every trial it evaluates."""

    def __init__(self, prob):
        self.prob = prob
        self.vals = []

    def eval(self, lam3, tangents=False):
        out, res = self.prob.eval(lam3, tangents=tangents)
        self.vals.append((float(res["Phi"][0]), float(res["rho"][0])))
        return out, res

    def lm_eval(self, mu3):
        r = self.prob.lm_eval(mu3)
        self.vals.append((float(r[2]), float(r[3])))
        return r


def has_near_tie(vals, eps, rel=TIE_REL):
    """True if a decision of the search on these trial values could flip under relative perturbations
    of size `rel`."""
    phi = np.array([v[0] for v in vals if np.isfinite(v[0])])
    rho = np.array([v[1] for v in vals if np.isfinite(v[1])])
    if rho.size and np.any(np.abs(rho - eps) <= rel * max(eps, 1e-300)):
        return True
    if phi.size > 1:
        s = np.sort(phi)
        gap = np.diff(s)
        if np.any(gap <= rel * np.maximum(np.abs(s[1:]), 1e-300)):
            return True
    return False
