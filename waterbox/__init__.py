"""Seeded synthetic inputs for the submatrix sign method.

This module only *builds inputs*: block-sparse symmetric matrices K in
block-compressed-sparse-column (BSC) form, their block sizes and the grouping
of block columns into submatrices.  It contains none of the method's
arithmetic (no gather, no sign function, no scatter, no reductions), so the
CPU oracle and the GPU path can both read what it produces without sharing
any code.

BSC layout (both triangles stored, block column J owns storage positions
``col_ptr[J] .. col_ptr[J+1]-1``; ``row_idx`` ascending within a column):
block (I, J) is a dense column-major ``blk_size[I] x blk_size[J]`` array,
placed at the running offset of the preceding blocks in storage order.  The
storage position doubles as the block's identifier, like the globally
sorted coordinate list of non-zero blocks in the paper (Sec. IV-A).

Water-like systems stand in for the paper's CP2K liquid-water benchmarks
(Sec. V: 32-molecule cells replicated NREP^3 times, atom-centred basis,
element truncation by eps_filter).  Here the truncation is a distance cutoff
(Sec. III-C: a finite R_max bounds the submatrix size), block sizes are
DZVP-like (O: 13, H: 5), and on-site energies alternate between -0.5 and
+0.5 Ha so that mu = 0 sits in a gap.
"""

from .systems import (  # noqa: F401
    BlockSparse,
    WATER_CONFIGS,
    water_system,
    water_config,
    dense_to_bsc,
    tb_chain,
    random_block_system,
    block_offsets,
)
