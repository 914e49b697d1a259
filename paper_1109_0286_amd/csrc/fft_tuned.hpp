// FFT plan variant per (precision, length, pass kind): 0 = E 16, 1 = E 8
// elements per thread (fft_device.hpp); rows per row-pass workgroup relative
// to the 64 KiB default.  Written by autotune.py from in-solve kernel timings
// on AMD Radeon Graphics; lengths not listed use variant 0, scale 1.
#pragma once

namespace fillk {

constexpr int tuned_fft_variant(bool f32, int n, int pass) {
  switch (n) {
    case 128: return f32 ? (pass == 0 ? 1 : 0)
                 : (pass == 0 ? 1 : 0);
    case 256: return f32 ? (pass == 0 ? 0 : 0)
                 : (pass == 0 ? 1 : 0);
    case 512: return f32 ? (pass == 0 ? 1 : 0)
                 : (pass == 0 ? 1 : 1);
    case 1024: return f32 ? (pass == 0 ? 1 : 1)
                 : (pass == 0 ? 1 : 1);
    case 2048: return f32 ? (pass == 0 ? 1 : 0)
                 : (pass == 0 ? 1 : 0);
    case 4096: return f32 ? (pass == 0 ? 0 : 1)
                 : (pass == 0 ? 0 : 0);
    default: return 0;
  }
}

constexpr int tuned_row_scale(bool f32, int n) {
  switch (n) {
    case 128: return f32 ? 2 : 2;
    case 256: return f32 ? 2 : 1;
    case 512: return f32 ? 1 : 1;
    case 1024: return f32 ? 1 : 1;
    case 2048: return f32 ? 1 : 1;
    case 4096: return f32 ? 2 : 2;
    default: return 1;
  }
}

}  // namespace fillk
