"""Growth-map surrogate: the library trains it and loads it; this module only passes the
configuration and holds the handles.

qs_surrogate_train (include/qs_surrogate.h) runs the whole pipeline on the device -- the
uniform-seed solver sweeps, the windowed growth targets, the example draws, the network's
training with AdamW and its held-out error table -- and writes one file; qs_surrogate_load
reads it back as a network and a device error table for qs_growth_map.
"""
from __future__ import annotations

from . import qs


def train(path, cfg=None, stream=None):
    """Train with the configuration dict `cfg` (keys of include/qs_surrogate.h; defaults for
    the rest) and write the result to `path`.  Returns the held-out statistics."""
    return qs.surrogate_train(path, cfg, stream)


def load(path, stream=None):
    """The trained surrogate in `path`: .net for qs_growth_map, .table the device address of
    its error table."""
    return qs.Surrogate(path, stream)
