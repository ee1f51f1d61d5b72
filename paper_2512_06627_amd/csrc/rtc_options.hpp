// hipRTC options of the specialized kernels, shared by the library's in-process compile and the
// compile helper program (paper_2512_06627_amd/rtc/fastlec_es_rtc.cpp), so that both produce the
// same code object for the same source.
#pragma once

namespace fes {
// Packed FP32 instructions are disabled for all device code.
inline const char* const kRtcOptions[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                                          "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int kRtcOptionCount = (int)(sizeof(kRtcOptions) / sizeof(kRtcOptions[0]));
}  // namespace fes
