// jit.cpp -- load-time specialisation of the net engine for one rule table.
//
// The device code (device.h) is compiled with hipRTC after the compiled rule
// templates have been written into it as constant arrays (namespace rt), so
// each rule's right-hand side becomes straight-line code (engine 3; engine 4
// is the same code with per-lane atomic reservations).  One code object per
// (rule table, device architecture, engine, engine width) holds the batch
// kernel and, for engine 3, the multi-workgroup engine of one net; it is
// built on first use and kept for the process.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/inet.h"
#include "inet_internal.h"
#include "runtime.h"

namespace inet {

extern const char *const kEmbeddedDeviceH;    // device.h, embedded at build time
extern const char *const kEmbeddedInternalH;  // inet_internal.h

namespace {

struct Module {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;   // the batch kernel
  hipFunction_t gfn = nullptr;  // the multi-workgroup engine of one net (engine 3)
  bool failed = false;
  std::string log;
};

std::mutex g_mu;
std::map<std::string, Module> g_mods;

std::string source_for(const CompiledRules &R, int engine, int wg, int qcap, int trace, int solo) {
  std::ostringstream o;
  o << "#define INET_STATIC_RULES 1\n#include \"inet_internal.h\"\n";
  o << "namespace inet { namespace rt {\n";
  o << "constexpr int NS = " << R.ns << ";\nconstexpr int NR = " << R.nr << ";\n";
  const int rows = R.nr > 0 ? R.nr : 1;
  o << "constexpr int T[" << rows << "][" << RT_WORDS << "] = {";
  for (int k = 0; k < rows; k++) {
    o << (k ? ",\n{" : "\n{");
    for (int w = 0; w < RT_WORDS; w++) {
      const int v = R.nr > 0 ? R.templ[(size_t)k * RT_WORDS + w] : 0;
      o << (w ? "," : "") << v;
    }
    o << "}";
  }
  o << "};\nconstexpr int ARITY[" << R.ns << "] = {";
  for (int i = 0; i < R.ns; i++) o << (i ? "," : "") << R.arity[i];
  o << "};\n} }\n#include \"device.h\"\n";
  const int maxl = R.max_links <= 4 ? 4 : MAXEQ;
  {
    LaunchShape sh = shape_for(wg, engine, R.max_links);
    sh.qcap = qcap;
    o << "extern \"C\" __global__ __launch_bounds__(" << wg << ") void inet_static_" << wg
      << "(const inet::NetDesc *__restrict__ d, const int *__restrict__ ord, int n, int *ctr,"
         " const int *__restrict__ r, int ns, int nr, unsigned ms, int flags, inet::KParams kp) {\n"
      << "  inet::reduce_body<" << wg << ", " << sh.qcap << ", " << engine << ", " << maxl
      << ", " << (trace ? "true" : "false") << ", " << solo
      << ">(d, ord, n, ctr, r, ns, nr, ms, flags, kp);\n}\n";
    if (engine == 3)
      o << "extern \"C\" __global__ __launch_bounds__(" << wg << ") void inet_grid_" << wg
        << "(const inet::NetDesc *__restrict__ d, const int *__restrict__ r, int ns, int nr,"
           " unsigned ms, int flags, inet::KParams kp) {\n"
        << "  inet::grid_body<" << wg << ", " << sh.qcap << ", " << maxl << ", "
        << (trace ? "true" : "false") << ", " << solo << ">(d, r, ns, nr, ms, flags, kp);\n}\n";
  }
  return o.str();
}

std::string key_for(const CompiledRules &R, const std::string &arch) {
  // FNV-1a over the device image of the rule table
  uint64_t h = 1469598103934665603ull;
  for (int32_t w : R.blob) {
    for (int b = 0; b < 4; b++) {
      h ^= (uint64_t)((w >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  }
  char buf[64];
  std::snprintf(buf, sizeof buf, "%016llx/", (unsigned long long)h);
  return std::string(buf) + arch;
}

// compile the specialised engine; code object into *code (no device needed)
int compile_code(const CompiledRules &R, const std::string &arch, int engine, int wg, int qcap,
                 int trace, int solo, std::vector<char> *code, std::string *log_out) {
  const std::string src = source_for(R, engine, wg, qcap, trace, solo);
  if (const char *dump = std::getenv("INET_JIT_DUMP")) {  // inspection aid
    if (FILE *f = std::fopen(dump, "w")) {
      std::fputs(src.c_str(), f);
      std::fclose(f);
    }
  }
  const char *headers[] = {kEmbeddedInternalH, kEmbeddedDeviceH};
  const char *names[] = {"inet_internal.h", "device.h"};
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "inet_static.hip", 2, headers, names) !=
      HIPRTC_SUCCESS)
    return INET_ENOSYS;
  const std::string archopt = "--offload-arch=" + arch;
  std::vector<const char *> opts = {archopt.c_str(), "-O3", "-std=c++17",
                                    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
                                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  size_t logn = 0;
  hiprtcGetProgramLogSize(prog, &logn);
  if (logn > 1) {
    std::vector<char> log(logn + 1, 0);
    hiprtcGetProgramLog(prog, log.data());
    log_out->assign(log.data());
  }
  if (cr != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return INET_ENOSYS;
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code->resize(n);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return INET_OK;
}

int build_module(const CompiledRules &R, const std::string &arch, int engine, int wg, int qcap,
                 int trace, int solo, Module *M) {
  std::vector<char> code;
  int rc = compile_code(R, arch, engine, wg, qcap, trace, solo, &code, &M->log);
  if (rc) return rc;
  if (hipModuleLoadData(&M->mod, code.data()) != hipSuccess) return INET_EHIP;
  const std::string name = "inet_static_" + std::to_string(wg);
  if (hipModuleGetFunction(&M->fn, M->mod, name.c_str()) != hipSuccess) return INET_EHIP;
  if (engine == 3) {
    const std::string gname = "inet_grid_" + std::to_string(wg);
    if (hipModuleGetFunction(&M->gfn, M->mod, gname.c_str()) != hipSuccess) return INET_EHIP;
  }
  return INET_OK;
}

}  // namespace

// Kernel of engine 3 or 4 for the rule table and engine width (built on first
// use); with `grid`, the multi-workgroup engine of one net (engine 3 only).
static int jit_kernel(const CompiledRules &R, int wg, int qcap, int engine, bool grid, int trace,
                      int solo, hipFunction_t *out) {
  if (engine != 3 && engine != 4) return INET_EINVAL;
  if (!shape_supported(wg) || (grid && engine != 3)) return INET_EINVAL;
  if (qcap < 64 || qcap > 8192 || (qcap & (qcap - 1)) || solo < 1 || solo > 4096) return INET_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return INET_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return INET_EHIP;
  std::string arch(prop.gcnArchName);
  const std::string key = key_for(R, arch) + "/" + std::to_string(dev) + "/" +
                          std::to_string(engine) + "/" + std::to_string(wg) + "/" +
                          std::to_string(qcap) + "/" + std::to_string(solo) +
                          (trace ? "/trace" : "");
  std::lock_guard<std::mutex> lock(g_mu);
  Module &M = g_mods[key];
  if (M.failed) return INET_ENOSYS;
  if (!M.mod) {
    int rc = build_module(R, arch, engine, wg, qcap, trace, solo, &M);
    if (rc) {
      M.failed = true;
      if (std::getenv("INET_JIT_LOG")) std::fprintf(stderr, "inet jit: %d\n%s\n", rc, M.log.c_str());
      return rc;
    }
  }
  *out = grid ? M.gfn : M.fn;
  return *out ? INET_OK : INET_EINVAL;
}

int jit_function(const CompiledRules &R, int wg, int engine, hipFunction_t *out) {
  const LaunchShape sh = shape_for(wg, engine, R.max_links);
  return jit_kernel(R, wg, sh.qcap, engine, false, 0, sh.solo, out);
}

int jit_launch(const CompiledRules &R, const LaunchShape &sh, int grid, const NetDesc *d,
               const int32_t *ord, int n, int32_t *ctr, const int32_t *r, uint32_t ms, int flags,
               const KParams &kp, hipStream_t s) {
  hipFunction_t f = nullptr;
  int rc = jit_kernel(R, sh.wg, sh.qcap, sh.engine, false, sh.trace, sh.solo, &f);
  if (rc) return rc;
  int ns = R.ns, nr = R.nr;
  KParams k = kp;
  void *args[] = {(void *)&d, (void *)&ord, (void *)&n, (void *)&ctr, (void *)&r,
                  (void *)&ns, (void *)&nr, (void *)&ms, (void *)&flags, (void *)&k};
  const unsigned dyn = (unsigned)(ns * ns + nr * RT_WORDS + ns) * 4;
  if (hipModuleLaunchKernel(f, grid, 1, 1, sh.wg, 1, 1, dyn, s, args, nullptr) != hipSuccess)
    return INET_EHIP;
  return INET_OK;
}

int jit_grid_launch(const CompiledRules &R, const LaunchShape &sh, int grid, const NetDesc *d,
                    const int32_t *r, uint32_t ms, int flags, const KParams &kp, hipStream_t s) {
  if (sh.engine != 3 || !kp.ctl) return INET_EINVAL;
  hipFunction_t f = nullptr;
  int rc = jit_kernel(R, sh.wg, sh.qcap, 3, true, sh.trace, sh.solo, &f);
  if (rc) return rc;
  int ns = R.ns, nr = R.nr;
  KParams k = kp;
  void *args[] = {(void *)&d, (void *)&r, (void *)&ns, (void *)&nr, (void *)&ms, (void *)&flags,
                  (void *)&k};
  const unsigned dyn = (unsigned)(ns * ns + nr * RT_WORDS + ns) * 4;
  if (hipModuleLaunchKernel(f, grid, 1, 1, sh.wg, 1, 1, dyn, s, args, nullptr) != hipSuccess)
    return INET_EHIP;
  return INET_OK;
}

static int occupancy_of(const CompiledRules &R, const LaunchShape &sh, bool grid, int *per_cu) {
  hipFunction_t f = nullptr;
  int rc = jit_kernel(R, sh.wg, sh.qcap, sh.engine, grid, sh.trace, sh.solo, &f);
  if (rc) return rc;
  const size_t dyn = (size_t)(R.ns * R.ns + R.nr * RT_WORDS + R.ns) * 4;
  return hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, sh.wg, dyn) == hipSuccess
             ? INET_OK
             : INET_EHIP;
}

int jit_occupancy(const CompiledRules &R, const LaunchShape &sh, int *per_cu) {
  return occupancy_of(R, sh, false, per_cu);
}

int jit_grid_occupancy(const CompiledRules &R, const LaunchShape &sh, int *per_cu) {
  if (sh.engine != 3) return INET_EINVAL;
  return occupancy_of(R, sh, true, per_cu);
}

}  // namespace inet

extern "C" int inet_jit_build(const inet_rules *rules, const char *arch, size_t *code_bytes,
                              char *log, size_t log_cap) {
  inet::CompiledRules R;
  int rc = inet::compile_rules(rules, &R);
  if (rc) return rc;
  if (!arch) return INET_EINVAL;
  // both specialised engines (3, then 4) at the default width (1024 lanes);
  // the first failure ends the build
  size_t total = 0;
  std::string msg;
  for (int engine = 3; engine <= 4 && rc == INET_OK; engine++) {
    std::vector<char> code;
    rc = inet::compile_code(R, arch, engine, 1024, inet::shape_for(1024, engine, R.max_links).qcap,
                            0, 64, &code, &msg);
    total += code.size();
  }
  if (log && log_cap) {
    std::strncpy(log, msg.c_str(), log_cap - 1);
    log[log_cap - 1] = 0;
  }
  if (code_bytes) *code_bytes = total;
  return rc;
}
