"""Seeded synthetic inputs (regular expressions and texts) shared by the tests,
the benchmark and the oracle.

This package holds no recognition arithmetic: it only draws random numbers and
writes bytes.  Whether a generated text is in the language is decided by the
oracle (or by the recognizer under test), never here.
"""

from .gen import (  # noqa: F401
    PCG,
    regexp_family,
    c1_regex,
    c1_texts,
    c2_regex_and_motifs,
    c2_texts,
    c3_regex,
    c3_texts,
    random_regex,
    random_text,
)
