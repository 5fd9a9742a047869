// Compile helper of libah: compiles one specialised scan program with hipRTC
// in a process of its own, so that several programs compile at the same time
// (hipRTC compiles one program at a time per process).  Touches no GPU.
//
//   ah_jitc <source file> <code object file> <compiler option>...
//
// Reads the HIP source, compiles it with the given options and writes the
// code object.  Exit status 0 on success; otherwise 1, with the compiler's log
// (or the failing step) written to the output file instead.
#include <hip/hiprtc.h>

#include <cstdio>
#include <string>
#include <vector>

namespace {

bool read_file(const char* path, std::string& out) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return false;
  char buf[1 << 16];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, n);
  std::fclose(f);
  return true;
}

bool write_file(const char* path, const char* data, size_t n) {
  FILE* f = std::fopen(path, "wb");
  if (!f) return false;
  const bool ok = std::fwrite(data, 1, n, f) == n;
  return std::fclose(f) == 0 && ok;
}

int fail(const char* out, const std::string& msg) {
  write_file(out, msg.data(), msg.size());
  return 1;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const char* in = argv[1];
  const char* out = argv[2];
  std::string src;
  if (!read_file(in, src)) return fail(out, "ah_jitc: cannot read the source");
  std::vector<const char*> opts(argv + 3, argv + argc);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "ah_scan.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(out, "ah_jitc: hiprtcCreateProgram failed");
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(out, "scan program failed to compile: " + log);
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  std::vector<char> code(n);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return write_file(out, code.data(), code.size()) ? 0 : 1;
}
