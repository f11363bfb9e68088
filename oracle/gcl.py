"""Parser for the paper's textual GCL genomes ("CONST 3.14; LOAD a:0; ADD; ...").

TEST INFRASTRUCTURE ONLY.  Token forms follow the GCL command table: CONST
carries a literal, LOAD carries ``label:index`` with a zero-based index.
COPY and PASTE carry a variable name ``@k``.  Produces the oracle's
interchange arrays (nodes, consts).  SQRT maps to the protected square root
(sqrt |a|) of the benchmark set.
"""
from __future__ import annotations

import numpy as np

from . import (ABS, ACOS, ADD, ASIN, ATAN, CBRT, CONST, COPY, COS, CUBE, DEL, DIV, DUP,
               EXP, LOAD, LOG, MUL, PASTE, POW, SIGN, SIN, SQRT, SQUARE, SUB, SWAP, TAN,
               TANH)

_NAMES = {"ADD": ADD, "SUB": SUB, "MUL": MUL, "DIV": DIV, "SIN": SIN,
          "COS": COS, "EXP": EXP, "LN": LOG, "SQRT": SQRT, "ABS": ABS,
          "DUP": DUP, "SWAP": SWAP, "DEL": DEL, "SQUARE": SQUARE, "POW": POW,
          "SIGN": SIGN, "CUBE": CUBE, "CBRT": CBRT, "TAN": TAN, "ARCSIN": ASIN,
          "ARCCOS": ACOS, "ARCTAN": ATAN, "TANH": TANH}


def parse(text):
    """Return (nodes uint32, consts float32) for one genome."""
    nodes, consts = [], []
    for tok in text.replace("\n", " ").split(";"):
        tok = tok.strip()
        if not tok:
            continue
        parts = tok.split()
        name = parts[0].upper()
        if name == "CONST":
            consts.append(np.float32(float(parts[1])))
            nodes.append(CONST | ((len(consts) - 1) << 8))
        elif name == "LOAD":
            idx = int(parts[1].split(":")[1])
            nodes.append(LOAD | (idx << 8))
        elif name in ("COPY", "PASTE"):
            k = int(parts[1].lstrip("@"))
            nodes.append((COPY if name == "COPY" else PASTE) | (k << 8))
        elif name in _NAMES:
            nodes.append(_NAMES[name])
        else:
            raise ValueError("unknown GCL command %r" % tok)
    return np.array(nodes, np.uint32), np.array(consts, np.float32)
