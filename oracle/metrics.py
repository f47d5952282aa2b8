"""Field-comparison metrics of Schrijver et al. (2006), as used for Table 1 of the paper.

TEST INFRASTRUCTURE (see the package docstring). B is the exact field, b the model, both [3, N].
  C_vec = sum B.b / sqrt(sum|B|^2 sum|b|^2)      C_cs = mean(B.b / (|B||b|))
  E'_n  = 1 - sum|b - B| / sum|B|                E'_m = 1 - mean(|b - B| / |B|)
  eps   = sum|b|^2 / sum|B|^2
"""
import numpy as np


def schrijver_metrics(B, b):
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    nB = np.sqrt(np.sum(B * B, axis=0))
    nb = np.sqrt(np.sum(b * b, axis=0))
    dot = np.sum(B * b, axis=0)
    diff = np.sqrt(np.sum((b - B) ** 2, axis=0))
    return dict(
        C_vec=float(np.sum(dot) / np.sqrt(np.sum(nB ** 2) * np.sum(nb ** 2))),
        C_cs=float(np.mean(dot / (nB * nb))),
        E_n=float(1.0 - np.sum(diff) / np.sum(nB)),
        E_m=float(1.0 - np.mean(diff / nB)),
        eps=float(np.sum(nb ** 2) / np.sum(nB ** 2)),
    )
