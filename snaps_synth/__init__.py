"""Seeded synthetic workloads for the SNAPS similarity self-join.

This package only draws random numbers and prepares inputs.  It holds none
of the method's arithmetic (no distances, neighbour searches, metrics or
ranks), so both the CPU oracle and the GPU path can consume its output
without sharing any code of the method.

The real inputs of the paper (the SNAPShot1 catalogue of 31,693 ZTF
asteroids and the LSST5M set derived from it, Sec. 2) are not available;
the generators below stand in for them with the shapes and distributions
described in the module docstring of :mod:`snaps_synth.generators`.
"""
from .generators import (  # noqa: F401
    ROOT_SEED,
    config_seeds,
    normalize_minmax,
    gen_c0,
    gen_isolated_fixture,
    snapshot1_like_raw,
    gen_c1,
    gen_c2,
    gen_c3_jobs,
    gen_c3_population,
    gen_c3_projected,
    load_c3_eps,
    gen_c4,
    all_masks,
    mask_features,
    load_c1_eps,
    load_c2_eps,
    load_c4_eps,
    FEATURE_NAMES,
    to_soa,
    C3Job,
    C4Request,
    C4Workload,
)
