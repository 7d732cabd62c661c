"""Seeded synthetic inputs for the oblique QR factorisation Z = QR, Q^T A Q = I.

This package only draws random numbers and builds test matrices with a
prescribed spectrum (the constructions of Section 7 of Lowery & Langou,
"Stability Analysis of QR factorization in an Oblique Inner Product").  It
holds none of the factorisation's arithmetic, so both the CPU oracle and the
GPU library can consume the very same arrays.
"""
from .gen import *  # noqa: F401,F403
