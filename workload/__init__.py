"""Seeded synthetic workloads for the guest-memory translate-and-copy path.

The generator builds, from a seed, everything both sides of a parity test
consume: each VM's guest-physical image (closed-form fill bytes with x86-64
page-table frames overlaid), its memslots, each process's page-table root,
the host-buffer pool bytes and the request descriptors with their epochs.
It holds none of the translation or copy arithmetic: page tables are
*encoded* from an explicit map of leaves, never walked.
"""
from .gen import (  # noqa: F401
    SPECS,
    Spec,
    Workload,
    REQ_DTYPE,
    SLOT_DTYPE,
    fill_bytes,
    make_workload,
    spec,
)
