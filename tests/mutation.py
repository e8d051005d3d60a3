"""Planting a mistake in a copy of an oracle module (CPU only).

A pin is only worth something if a plausible mistake in the oracle makes it fail.
``mutated(module, (old, new), ...)`` returns a fresh module object built from the
source text of ``module`` with each ``old`` snippet replaced by ``new`` (every snippet
must occur exactly once, so a stale mutation fails loudly instead of silently testing
the unmutated code).  The original module is left untouched.
"""
from __future__ import annotations

import inspect
import itertools
import sys
import types

_count = itertools.count()


def mutated(module, *replacements) -> types.ModuleType:
    src = inspect.getsource(module)
    for old, new in replacements:
        n = src.count(old)
        if n != 1:
            raise AssertionError(f"mutation target {old!r} occurs {n} times in {module.__name__}")
        src = src.replace(old, new)
    name = f"{module.__name__}_mutant{next(_count)}"
    m = types.ModuleType(name)
    m.__dict__["__package__"] = module.__package__
    sys.modules[name] = m  # dataclasses look their module up by name
    try:
        exec(compile(src, f"<mutant of {module.__name__}>", "exec"), m.__dict__)
    finally:
        del sys.modules[name]
    return m
