"""Seeded synthetic inputs shared by the HIP path and the oracle.

Holds random gauge fields, Gaussian sources and rational-approximation
coefficients only; nothing here performs the solver's arithmetic.
"""
from .gauge import (GELL_MANN, GENERATORS, check_dims, gaussian_block, random_gauge,
                    random_gauge_transform, unit_gauge, volume)
from .rational import RationalApprox, remez, zolotarev_inv_sqrt
