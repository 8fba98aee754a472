"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2411_18370_amd``) and never imports it; the only module both sides use
is the seeded input generator ``paper_2411_18370_amd.synth``, which holds no
arithmetic of the method.

``ft_oracle.c`` holds the statistic itself (bins, sums, z, toplists);
``inject.py`` the signal model used to plant injections into test tables,
``bank.py`` the random template bank of sources in binary systems and
``mlp.py`` the FP64 network used to check the surrogate's kernels.
"""
from .core import (  # noqa: F401
    build, lib_path, bins_list, eval_list, eval_grid, noise_moments, critical_ratio,
    subband, toplist, grid_params, pcos, bins_binary, eval_binary,
)
