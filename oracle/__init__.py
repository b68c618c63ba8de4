"""CPU oracle for batched 3D Gaussian Splatting of rigid-body environments.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path.

What it computes (the paper renders its environments with standard 3D Gaussian
Splatting built on gsplat, Sec. "Batch Renderer Optimization", and poses
Gaussian clusters with their rigid bodies, "Rigid-Link Gaussian Kinematics"):

* ``spec32.bin_ref``   -- the binning decisions (cull set, depth-key bits,
  tile rectangles, sorted (key, Gaussian) lists and tile ranges) under an
  IEEE binary32 specification with one rounding per operation and no FMA, so
  that a GPU implementation can match them bit for bit.
* ``attrs64.attrs64``  -- the continuous per-Gaussian quantities (projected
  mean, conic, colour from spherical harmonics, depth, opacity) in float64,
  written as the plain EWA/3DGS definitions.
* ``render.render_ref`` -- per-pixel front-to-back alpha compositing in float64
  over the tile lists (C, ``composite.c``), with alternative results where a
  threshold decision lies within rounding distance of its boundary.
* ``brute.brute_ref``  -- every Gaussian at every pixel in (depth, index)
  order; for tiny scenes only.
* ``observe``          -- the observation epilogue (exposure gain, contrast,
  brightness, clamp, u8 / f16 pixels) applied to oracle colours.
* ``lidar.lidar_ref``   -- batch LiDAR: every ray against every Gaussian in
  float64 (peak response along the ray), composited in centre-distance order.
"""
from .spec32 import bin_ref, quat_to_rot32  # noqa: F401
from .attrs64 import attrs64  # noqa: F401
from .render import render_ref, composite64, oracle_threads, set_oracle_threads  # noqa: F401
from .brute import brute_ref  # noqa: F401
from .observe import observe64, observe32, observe_codes, quantise_u8  # noqa: F401
from .lidar import lidar_ref, lidar_ray_variants, ray_directions  # noqa: F401
