"""Seeded synthetic inputs for Fourier-slice insertion.

Shared by the tests, the benchmark and the smoke check; it holds none of the
insertion arithmetic (no blob, no gather, no scatter).  It draws orientations
and Gaussian phantoms, computes the exact line-integral projections of the
phantom in each orientation and their centered 2D DFTs in Hermitian half-plane
layout, which is the input form of the insertion step.
"""
from .phantom import (  # noqa: F401
    Phantom,
    Workload,
    clustered_quaternions,
    make_phantom,
    make_slices,
    make_workload,
    project,
    random_quaternions,
    slices_from_projections,
    phantom_ft,
    WORKLOADS,
    BATCHES,
    batch_specs,
    batch_quaternions,
)
