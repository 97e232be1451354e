"""Parameter sets of the fixed-point RBF support-vector regressor (Sec. 3.4).

A model is a dict of integer arrays:
  sv        [n_sv, 5] int32   support vectors in the 10-bit feature space
  beta      [n_sv]    int32   dual coefficients, Q20
  beta0     int              intercept, Q40
  feat_lo   [5]       int64  per-feature offset of the integer affine map
  feat_mul  [5]       int64  per-feature multiplier (Q16) of that map
  g_mul     int              kernel-width multiplier (Q32)
  table     [1024]    int32  kernel values exp(-(i + 1/2) / 64), Q20
  theta     [3]       int64  thresholds of the 4-, 8- and 12-bit choices, Q40

This module only draws such parameter sets (for tests) and builds the kernel
table; it never evaluates a model.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 5
U_MAX = 1023
TABLE_N = 1024
TABLE_PER_UNIT = 64      # table entries per unit of gamma * ||du||^2
Q_BETA = 20
Q_TABLE = 20


def rbf_table(n=TABLE_N, per_unit=TABLE_PER_UNIT, q=Q_TABLE):
    i = np.arange(n, dtype=np.float64)
    return np.rint(np.exp(-(i + 0.5) / per_unit) * (1 << q)).astype(np.int32)


def gamma_to_gmul(gamma):
    """Q32 multiplier mapping sum((du)^2) on the 0..1023 grid to a table index."""
    return int(np.rint(gamma * TABLE_PER_UNIT / (U_MAX ** 2) * 2.0 ** 32))


def random_model(seed, n_sv, feat_lo, feat_mul, gamma=1.0, beta_scale=0.5,
                 theta=(-0.2, 0.0, 0.2)):
    """A seeded model with random support vectors and coefficients."""
    r = np.random.Generator(np.random.PCG64([seed, 991]))
    sv = r.integers(0, U_MAX + 1, size=(n_sv, N_FEAT)).astype(np.int32)
    beta = np.rint(r.uniform(-beta_scale, beta_scale, size=n_sv) * (1 << Q_BETA))
    return dict(
        n_sv=int(n_sv), sv=sv, beta=beta.astype(np.int32),
        beta0=int(np.rint(r.uniform(-0.1, 0.1) * 2.0 ** 40)),
        feat_lo=np.asarray(feat_lo, dtype=np.int64),
        feat_mul=np.asarray(feat_mul, dtype=np.int64),
        g_mul=gamma_to_gmul(gamma), table=rbf_table(),
        theta=np.rint(np.asarray(theta, dtype=np.float64) * 2.0 ** 40).astype(np.int64),
    )
