// Compile helper: one hipRTC compile of a specialized-kernel program in a process of its own.
//
// hipRTC serializes compiles inside one process (four threads take as long as four compiles in
// a row), so the library compiles the programs of a grouped compile in child processes running
// this program, side by side.  It needs no GPU and links hipRTC only.
//
// Usage: fastlec_es_rtc <source file> <code object file>
// Exit status 0 with the code object written; otherwise non-zero with hipRTC's log on stderr.
// The code object is written to "<code object file>.part" and renamed when complete, so the
// file under its own name is always whole.
#include <hip/hiprtc.h>

#include <cstdio>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "../csrc/rtc_options.hpp"

int main(int argc, char** argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: fastlec_es_rtc <source> <code object>\n");
        return 2;
    }
    std::ifstream in(argv[1], std::ios::binary);
    if (!in) {
        std::fprintf(stderr, "fastlec_es_rtc: cannot read %s\n", argv[1]);
        return 2;
    }
    const std::string src((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "fes_es_kernel.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        std::fprintf(stderr, "fastlec_es_rtc: hiprtcCreateProgram failed\n");
        return 1;
    }
    if (hiprtcCompileProgram(prog, fes::kRtcOptionCount, fes::kRtcOptions) != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        std::fprintf(stderr, "%s\n", log.c_str());
        hiprtcDestroyProgram(&prog);
        return 1;
    }
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    std::vector<char> code(size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    const std::string part = std::string(argv[2]) + ".part";
    {
        std::ofstream out(part, std::ios::binary);
        out.write(code.data(), (std::streamsize)code.size());
        out.close();
        if (!out) {
            std::fprintf(stderr, "fastlec_es_rtc: cannot write %s\n", part.c_str());
            std::remove(part.c_str());
            return 1;
        }
    }
    if (std::rename(part.c_str(), argv[2]) != 0) {
        std::fprintf(stderr, "fastlec_es_rtc: cannot rename %s\n", part.c_str());
        std::remove(part.c_str());
        return 1;
    }
    return 0;
}
