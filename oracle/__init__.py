"""CPU oracle for the Mixture Graph box-histogram path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package. It shares no code with the HIP library (``paper_2009_02702_amd``):
it compacts IDs, clips boxes, builds mipmaps and decomposes boxes on its own.

What each module follows (sections, equations, figures and tables of
Al-Thelaya, Agus, Schneider, "The Mixture Graph", IEEE VIS 2020):

- ``scan``       O1, the ground truth: brute-force level-0 box histograms
                 (uint64 counts, fp64 fractions), C + OpenMP, plus a NumPy
                 ``bincount`` form for cross-checks. Definition of a histogram
                 over a sub-volume (Sec. "Fast Sub-Volume Queries").
- ``mipmap``     the normalized histogram mipmap of Eq. (mip) (Sec.
                 "Normalized Histogram Mipmap"), written out from the level-0
                 volume, per level and voxel.
- ``footprint``  the footprint assembly of the appendix algorithm "Footprint
                 assembly in 3D" (1D aligned power-of-two steps per axis,
                 tensor product, tessellation by cubes of the smallest side),
                 and a brute-force maximal aligned-cube decomposition.
- ``tf``         per mip voxel, the mean transfer-function colour over its
                 level-0 support: what the colour palette of a node must hold
                 (Sec. "Reconstruction", Sec. "Rendering").
- ``dag``        exact (rational) and fp64 forward expansion and reverse push
                 over a given binary-lerp DAG (Sec. "Factorization", Figs.
                 "factorization", "tree", "DAG"); used as a diagnostic on
                 graphs the library builds and on the paper's own example.
"""
from . import dag, footprint, mipmap, scan, tf  # noqa: F401
