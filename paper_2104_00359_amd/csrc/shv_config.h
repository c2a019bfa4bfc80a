// Launch-shape constants shared by host and device code.
#pragma once

#define SHV_BLOCK 256                              // threads per block (4 waves of 64)
#define SHV_WAVES_PER_BLOCK (SHV_BLOCK / 64)
#define SHV_MAX_CHUNK 512                          // spheres per block in the pair kernels (LDS bound)
#define SHV_MAX_CHANNELS 4                         // colour channels per multi-channel shading call
#define SHV_ENV_MAX_ROWS 64                         // map rows per block of the environment-map projection
