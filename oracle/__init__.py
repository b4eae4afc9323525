"""FP64 CPU oracle (test infrastructure only; see rl_oracle's header)."""
from .rl_oracle import (  # noqa: F401
    EPS, dft_matrix, dft3, idft3, psf_centre, check_psf, centred_kernel, otf,
    forward, adjoint, conv3d, conv_direct, corr_direct, conv_direct_at,
    ratio, loglik, rl, rl_direct, rel_l2,
)
from .accel_oracle import extrapolate, rl_accel  # noqa: F401,E402
from .boundary_oracle import (  # noqa: F401,E402
    embed_kernel, conv_periodic, corr_periodic, conv_zero, corr_zero, conv_zero_at, rl_general,
)
from .stop_oracle import psnr_si, rel_change, rl_stop  # noqa: F401,E402
from .fsc_oracle import fsc, fsc_sums, resolution, split_diagonal  # noqa: F401,E402
from .ssim_oracle import ssim  # noqa: F401,E402
