"""Seeded synthetic inputs for the failure-less Aho-Corasick (PFAC) matcher.

This package only draws random keywords, texts, planted copies and request
traces.  It holds none of the matching arithmetic: both the CPU oracle and the
GPU library consume what it produces, and neither imports the other.
"""

from .gen import (  # noqa: F401
    KeywordSpec,
    Workload,
    BatchWorkload,
    ServedWorkload,
    SPECS,
    make_keywords,
    make_text,
    plant,
    keywords_to_csr,
    config_tiny,
    config_sweep,
    config_large_automaton,
    config_batched,
    config_served,
    paper_workload,
    SWEEP_SIZES,
    KIB,
    MIB,
    GIB,
)
