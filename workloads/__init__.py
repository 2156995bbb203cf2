"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds input generation only (mechanism files and state fields);
it performs none of the integration arithmetic.
"""
from __future__ import annotations

import pathlib

MECH_DIR = pathlib.Path(__file__).resolve().parent / "mech"

# Workloads: sizes, step and tolerances.  Seeds are fixed here.
WORKLOADS = {
    # independent cells, uniform draw; the small parity case
    "uniform4k": dict(mech="m9", kind="uniform", n=4096, seed=100,
                      dt=1e-8, rtol=1e-8, atol=1e-12),
    # 1024 x 1024 RDE-shaped field; the headline workload
    "rde1m": dict(mech="m9", kind="rde", width=1024, height=1024, seed=101,
                  dt=5e-9, rtol=1e-8, atol=1e-12),
    # 64 fields, log-uniform 1e4..2e6 cells, RDE-shaped; two mechanisms
    "amr64": dict(mechs=("m9", "m13"), kind="fields", n_fields=64, seed=102,
                  dt=5e-9, rtol=1e-8, atol=1e-12),
    # 512 x 512 RDE-shaped field for the adjoint
    "adj256k": dict(mech="m9", kind="rde", width=512, height=512, seed=103,
                    dt=1e-8, rtol=1e-8, atol=1e-12, t_ref=1000.0),
    # 2048 x 2048 RDE-shaped field, 32-species mechanism
    "big4m": dict(mech="m32", kind="rde", width=2048, height=2048, seed=104,
                  dt=5e-9, rtol=1e-8, atol=1e-12),
}


def mech_path(name: str) -> str:
    return str(MECH_DIR / f"{name}.mech")


def mech_text(name: str) -> str:
    return (MECH_DIR / f"{name}.mech").read_text()
