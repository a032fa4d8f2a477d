// Runtime dtype / SH-order / MLP-mode dispatch onto the compiled kernel instances.
#pragma once

#define PSDF_MLP_SWITCH(mlp_dt, ...)                                  \
  switch (mlp_dt) {                                                   \
    case 0: { constexpr int M = ::psdf::MLP_F32; __VA_ARGS__; break; }  \
    case 1: { constexpr int M = ::psdf::MLP_F16; __VA_ARGS__; break; }  \
    case 2: { constexpr int M = ::psdf::MLP_BF16; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;                             \
  }

#define PSDF_SH_SWITCH(n_sh, ...)                              \
  switch (n_sh) {                                              \
    case 1: { constexpr int NSH = 1; __VA_ARGS__; break; }     \
    case 4: { constexpr int NSH = 4; __VA_ARGS__; break; }     \
    case 9: { constexpr int NSH = 9; __VA_ARGS__; break; }     \
    case 16: { constexpr int NSH = 16; __VA_ARGS__; break; }   \
    default: return hipErrorInvalidValue;                      \
  }

#define PSDF_DT_SWITCH(sdf_dt, feat_dt, ...)                                                      \
  if (sdf_dt == 0 && feat_dt == 0) { typedef float ST; typedef float FT; __VA_ARGS__; }           \
  else if (sdf_dt == 0 && feat_dt == 1) { typedef float ST; typedef _Float16 FT; __VA_ARGS__; }   \
  else if (sdf_dt == 1 && feat_dt == 1) { typedef _Float16 ST; typedef _Float16 FT; __VA_ARGS__; } \
  else if (sdf_dt == 1 && feat_dt == 0) { typedef _Float16 ST; typedef float FT; __VA_ARGS__; }   \
  else return hipErrorInvalidValue;
