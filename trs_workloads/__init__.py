"""Seeded synthetic inputs for the term-rewriting hot path.

This package holds only input preparation: the rewrite systems as text, a
parser that turns that text into the integer encoding the C-ABI and the oracle
both accept, and seeded generators for the ground input terms.  It performs no
rewriting, matching or normalisation of any kind, so that the oracle and the
GPU path share nothing but their inputs.
"""

from .trs_text import TRS, parse_trs, encode_term, decode_prefix, term_to_str
from . import systems, generators

__all__ = ["TRS", "parse_trs", "encode_term", "decode_prefix", "term_to_str",
           "systems", "generators"]
