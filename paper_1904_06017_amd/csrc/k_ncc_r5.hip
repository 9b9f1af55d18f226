// NCC cost kernels (Eq. 8) instantiated for block radius r = 5.
#include "ncc_impl.h"

namespace stereo {
hipError_t launch_ncc_r5(const Plan& P, const void* ref, const float* tar_w, const float* zX,
                         const float* isdX, const float* zY, const float* isdY, float* C,
                         int out_w, int64_t out_pitch, int64_t out_slice, int anchor,
                         int d_first, int d_end, int quad, int pad, hipStream_t s, float* C2) {
  if (P.p.dtype == STEREO_U8)
    return launch_ncc_r<5, uint8_t>(P, (const uint8_t*)ref, tar_w, zX, isdX, zY, isdY, C, out_w,
                                     out_pitch, out_slice, anchor, d_first, d_end, quad, pad, s,
                                     C2);
  return launch_ncc_r<5, float>(P, (const float*)ref, tar_w, zX, isdX, zY, isdY, C, out_w,
                                 out_pitch, out_slice, anchor, d_first, d_end, quad, pad, s, C2);
}
hipError_t launch_ncc_jobs_r5(stereo_dtype dt, int quad, int dc, const NccJob* jobs,
                              const int* first, int n, int blocks, char* base, hipStream_t s) {
  if (dt == STEREO_U8) return ncc_jobs_r<5, uint8_t>(quad, dc, jobs, first, n, blocks, base, s);
  return ncc_jobs_r<5, float>(quad, dc, jobs, first, n, blocks, base, s);
}
}  // namespace stereo
