"""MI355X-native all-pairs hot path (Rocket, arXiv 2009.04755).

For n items and a pair function f, computes f(a_i, a_j) for every pair i < j
(Section III) on one gfx950 GPU: items are pre-processed once, the pair matrix is
split divide-and-conquer into tiles (Section IV-B), and a persistent kernel pulls
tiles from an on-device queue while item tiles sit in LDS/registers.  The work is
done by hand-written HIP kernels behind the C ABI in ``include/rocket.h``; this
package is a thin ctypes binding (``api``) plus seeded input generators
(``synth``).
"""
from .api import (Clouds, Context, OverlapCost, SparseSet, allpairs, allpairs_noalloc, default_context,  # noqa: F401
                  num_pairs, pair_index, plan_tiles, probe_valu, register)
