"""The oracle: test infrastructure, never part of the product path.

Plain, slow, FP64 CPU implementations of what the GPU library computes, written
from the paper (Sitaru & Gekle, arXiv 2109.04455) and pinned by the CPU tests:

* ``lbref``        -- C, single-threaded: D2Q9 BGK flow, D2Q5 ADR with link or
                      node reactions, outlet fluxes and efficiency.
* ``torch_ref``    -- the same ADR step in plain PyTorch-CPU FP64 ops, for
                      gradients by autograd (reference for the adjoint).
* ``steady_direct``-- the ADR step assembled as a sparse affine map and solved
                      for its fixed point (and its adjoint) directly.
* ``rwpt``         -- an independent random-walk particle tracker.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with
``paper_2109_04455_amd`` and imports nothing from it.
"""
