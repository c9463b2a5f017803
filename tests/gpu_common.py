"""Shared helpers of the GPU tests: oracle builds (cached per process) and
slot mapping between the library and the oracle."""
import sys

import numpy as np

import synth
from oracle.dh2 import OracleDH2

_oracles = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_for(name, norm="fro"):
    key = (name, norm)
    if key not in _oracles:
        w = synth.WORKLOADS[name]
        V, T = synth.make_mesh(w)
        _oracles[key] = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, norm=norm)
    return _oracles[key]


def build_handle(name, **kw):
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    say("[gpu] dh2_build workload=%s n=%d kappa=%g m=%d leaf=%d eta=%g eta1=%g tol=%g"
        % (name, len(T), w.kappa, w.order, w.leaf, w.eta, w.eta1, w.tol))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, **kw)
    slots = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1).export()["slots"]
    return h, slots


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
