"""MI355X-native (gfx950) implementation of the CentRA hot path.

CentRA (Pellegrina, "Efficient Centrality Maximization with Rademacher
Averages", KDD 2023) approximates set-betweenness centrality maximisation
by progressive sampling of shortest paths, greedy max coverage and a
Monte-Carlo Rademacher bound.  The hot path runs in the HIP kernels of
libcentra.so behind the C ABI of include/centra.h; `binding` exposes the
same entry points to Python (argument marshalling only).  `inputs` holds
the seeded synthetic workload generators.
"""
from . import binding  # noqa: F401  (the library itself is loaded on first use)
