"""MI355X (gfx950) LiDAR depth densification: nearest-depth projection and
RGB-guided joint bilateral filtering (arXiv 2601.01210), as hand-written HIP
kernels behind the C ABI in include/jbfd.h.

The Python layer only marshals arguments (torch tensors for device memory
and streams) into the C library; every step of the computation runs in the
HIP kernels. There is no CPU fallback: if libjbfd.so is missing the calls
raise.
"""
from .binding import (BatchView, JbfdError, Precision,  # noqa: F401
                      abi_version, backproject, backproject_ws_bytes,
                      batch_check, batch_run, batch_table_bytes,
                      remove_occluded, batch_upload, densify, densify_backward,
                      densify_prepare, densify_two_stage, densify_workspace,
                      densify_ws_bytes, library_path, motion_mask, pool3,
                      project, project_densify, project_densify_noalloc,
                      project_motion, restore_merge, two_stage_ws_bytes,
                      zbuf_clear)
