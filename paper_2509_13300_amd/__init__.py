"""MI355X-native degenerate-primer scan, melting temperature and amplicon
calling (AmpliconHunter's hot path, arXiv 2509.13300).

The work runs in libah.so (include/ah.h): hand-written HIP kernels for gfx950
plus a per-primer-set specialised scan kernel.  ``_lib`` is the ctypes
binding with the C names; ``path`` a thin driver that allocates buffers with
torch and calls the entry points in order.
"""
from . import _lib  # noqa: F401
from ._lib import (ah_pack_genomes, ah_pack_layout, ah_pair_amplicons, ah_scan_primers,  # noqa: F401
                   ah_tm)

__all__ = ["ah_pack_layout", "ah_pack_genomes", "ah_scan_primers", "ah_tm", "ah_pair_amplicons"]
