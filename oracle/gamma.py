"""Euclidean Dirac matrices used by the oracle (test infrastructure only).

Eq. 3 of the paper uses gamma_mu without fixing a basis.  The oracle uses the
chiral (DeGrand-Rossi) basis written out explicitly below: Hermitian,
{gamma_mu, gamma_nu} = 2 delta_{mu nu}, gamma_5 = gamma_1 gamma_2 gamma_3
gamma_4 = diag(1, 1, -1, -1).  Rows and columns run over spin 0..3.
"""
import numpy as np

_i = 1j

GAMMA = np.array(
    [
        [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],  # gamma_1
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],  # gamma_2
        [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],  # gamma_3
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],  # gamma_4
    ],
    dtype=np.complex128,
)

GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)

ID4 = np.eye(4, dtype=np.complex128)
