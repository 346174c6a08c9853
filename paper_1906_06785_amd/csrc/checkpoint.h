// Checkpoint files of a TT pair (host side; format in checkpoint.cpp).
#pragma once

namespace sgtt {
// dims: per TT (velocity, pressure) n1, n2, n3, r1, r2; cores: core 1, 2, 3
// of the velocity TT, then of the pressure TT, compact (ld = live rank).
int pair_file_write(const char* path, const int* dims, const double* const* cores);
int pair_file_info(const char* path, int* dims);
// caps: per TT n1, n2, n3, cap1, cap2 of the destination buffers
int pair_file_read(const char* path, const int* caps, double* const* cores, int* dims);
// parameter files of a network with n inputs and outputs and hidden width w
// (nparam = w n + w + w w + w + n w + n FP32 values)
int net_file_write(const char* path, int n, int w, long nparam, const float* params);
int net_file_info(const char* path, int* n, int* w, long* nparam);
int net_file_read(const char* path, int n, int w, float* params);
}  // namespace sgtt
