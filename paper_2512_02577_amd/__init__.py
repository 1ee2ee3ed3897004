"""MI355X (gfx950) implementation of the local p-multigrid vertex-patch smoother inside an
h-multigrid preconditioned flexible CG for the high-order Q_p Laplacian.

The compute path is libpmg.so (HIP kernels behind the C interface in include/pmg.h);
`paper_2512_02577_amd.pmg` is its Python binding and `paper_2512_02577_amd.inputs` holds
the seeded synthetic inputs.  Importing this package loads nothing native.
"""
