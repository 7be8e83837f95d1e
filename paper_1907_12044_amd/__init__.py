"""MI355X-native one-site TDVP-PS (projector-splitting TD-DMRG) on HIP/gfx950.

The compute path is libtdvp.so (HIP kernels + C ABI, include/tdvp.h); this
package is its thin Python binding.
"""

from .tdvp import (  # noqa: F401
    FP32,
    FP64,
    AU_PER_FS,
    HARTREE_PER_CM,
    Context,
    DeviceEnvs,
    DeviceMpo,
    DeviceMps,
    PsEnsemble,
    PsRun,
    TdvpError,
    env_update,
    envs_build,
    fmo_model,
    heff_apply,
    holstein_mpo,
    lanczos_expm,
    lib,
    observe,
    ps_step,
    qr,
    right_canonicalize,
    workspace_bytes,
)
