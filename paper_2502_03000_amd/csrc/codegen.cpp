// Element-wise kernels generated per expression.
//
// The paper fuses an element-wise expression by having the C++ compiler
// instantiate a loop tailored to that expression at compile time (Sec. II,
// the Z[i] = 0.4*X[i] + 0.6*Y[i] loop). Here the expression is known when
// the plan is made, so plan time plays the role of compile time: the
// post-order program is turned into straight-line HIP source (one register
// per intermediate, no interpreter dispatch, no stack traffic), compiled for
// gfx950 with hipRTC, loaded as a module and cached by source text. Each
// lane evaluates one 16-byte pack of every operand (one-shot grid,
// non-temporal loads and stores: a pure stream through HBM).
//
// When hipRTC is unavailable, or an operand is not dense and 16-byte
// aligned, the interpreter kernel runs instead (same program, same result
// up to the order of rounding, which is identical here: both evaluate the
// same operations in the same order per element).
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace hexla {

namespace {

std::mutex g_mu;
struct Compiled {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  std::string err;
};
std::map<std::string, Compiled> g_cache;  // key: device + source

std::string lit(double c, bool f32) {
  char buf[64];
  if (f32) std::snprintf(buf, sizeof buf, "%af", float(c));
  else std::snprintf(buf, sizeof buf, "%a", c);
  return buf;
}

}  // namespace

bool codegen_enabled() {
  const char* e = std::getenv("HEXLA_CODEGEN");
  return !(e && e[0] == '0');
}

// HIP source of the generated kernel for program p over n_leaf operands.
std::string codegen_source(const EwHost& p, int dtype) {
  const bool f32 = dtype == HEXLA_F32;
  const char* T = f32 ? "float" : "double";
  const int V = f32 ? 4 : 2;
  const int nl = int(p.leaves.size());
  std::ostringstream s;
  s << "typedef " << T << " vT __attribute__((ext_vector_type(" << V << ")));\n";
  s << "extern \"C\" __global__ void __launch_bounds__(256) hexla_ew(";
  for (int l = 0; l < nl; ++l) s << "const " << T << "* __restrict__ p" << l << ", ";
  s << T << "* __restrict__ out, long n_pack, long n_total) {\n";
  s << "  const long q = (long)blockIdx.x * 256 + threadIdx.x;\n";
  // body: straight-line evaluation of one element, given leaf values x<l>
  std::ostringstream body;
  std::vector<std::string> st;
  int tmp = 0;
  auto fresh = [&]() { return "t" + std::to_string(tmp++); };
  for (int i = 0; i < p.n_instr; ++i) {
    const int op = p.op[i], a = p.arg[i];
    std::string r;
    switch (op) {
      case k::EW_LEAF: st.push_back("x" + std::to_string(a)); continue;
      case k::EW_CONST: st.push_back("(" + std::string(T) + ")" + lit(p.cst[a], f32)); continue;
      case k::EW_EXTRA:
      case k::EW_IDENT: return std::string();  // not generated
      default: break;
    }
    r = fresh();
    if (op >= k::EW_ADD && op <= k::EW_RDIV) {
      const std::string rhs = st.back();
      st.pop_back();
      const std::string lhs = st.back();
      st.pop_back();
      const char* sym = op == k::EW_ADD ? "+" : (op == k::EW_SUB || op == k::EW_RSUB) ? "-"
                      : op == k::EW_MUL ? "*" : "/";
      const bool rev = op == k::EW_RSUB || op == k::EW_RDIV;
      body << "      const " << T << " " << r << " = " << (rev ? rhs : lhs) << " " << sym << " "
           << (rev ? lhs : rhs) << ";\n";
    } else {
      const std::string x = st.back();
      st.pop_back();
      switch (op) {
        case k::EW_NEG: body << "      const " << T << " " << r << " = -" << x << ";\n"; break;
        case k::EW_EXP:
          body << "      const " << T << " " << r << " = " << (f32 ? "expf(" : "exp(") << x << ");\n";
          break;
        case k::EW_SCALE:
          body << "      const " << T << " " << r << " = " << x << " * (" << T << ")" << lit(p.cst[a], f32) << ";\n";
          break;
        case k::EW_ADDC:
          body << "      const " << T << " " << r << " = " << x << " + (" << T << ")" << lit(p.cst[a], f32) << ";\n";
          break;
        case k::EW_LEAFMUL:
          body << "      const " << T << " " << r << " = " << x << " * x" << a << ";\n";
          break;
        case k::EW_LEAFADD:
          body << "      const " << T << " " << r << " = " << x << " + x" << a << ";\n";
          break;
        default: return std::string();
      }
    }
    st.push_back(r);
  }
  if (st.size() != 1) return std::string();
  const std::string result = st.back();
  s << "  if (q < n_pack) {\n";
  for (int l = 0; l < nl; ++l)
    s << "    const vT v" << l << " = __builtin_nontemporal_load((const vT*)p" << l << " + q);\n";
  s << "    vT res;\n#pragma unroll\n    for (int e = 0; e < " << V << "; ++e) {\n";
  for (int l = 0; l < nl; ++l) s << "      const " << T << " x" << l << " = v" << l << "[e];\n";
  s << body.str() << "      res[e] = " << result << ";\n    }\n";
  s << "    __builtin_nontemporal_store(res, (vT*)out + q);\n  } else {\n";
  s << "    const long t = n_pack * " << V << " + (q - n_pack);\n    if (t < n_total) {\n";
  for (int l = 0; l < nl; ++l) s << "      const " << T << " x" << l << " = p" << l << "[t];\n";
  s << body.str() << "      out[t] = " << result << ";\n    }\n  }\n}\n";
  return s.str();
}

// Returns the compiled kernel for (device, source), compiling on first use.
hipFunction_t codegen_get(int device, const std::string& src, std::string* err) {
  if (src.empty()) {
    if (err) *err = "program not generated";
    return nullptr;
  }
  const std::string key = std::to_string(device) + "\n" + src;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    if (err) *err = it->second.err;
    return it->second.fn;
  }
  Compiled c;
  hiprtcProgram prog = nullptr;
  if (hiprtcCreateProgram(&prog, src.c_str(), "hexla_ew.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    c.err = "hiprtcCreateProgram failed";
  } else {
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 6, opts);
    if (r != HIPRTC_SUCCESS) {
      size_t n = 0;
      hiprtcGetProgramLogSize(prog, &n);
      std::string log(n, '\0');
      if (n) hiprtcGetProgramLog(prog, &log[0]);
      c.err = std::string("hipRTC: ") + hiprtcGetErrorString(r) + " " + log;
    } else {
      size_t n = 0;
      hiprtcGetCodeSize(prog, &n);
      std::vector<char> code(n);
      hiprtcGetCode(prog, code.data());
      hipError_t e = hipModuleLoadData(&c.mod, code.data());
      if (e == hipSuccess) e = hipModuleGetFunction(&c.fn, c.mod, "hexla_ew");
      if (e != hipSuccess) {
        c.err = std::string("module load: ") + hipGetErrorString(e);
        c.fn = nullptr;
      }
    }
    hiprtcDestroyProgram(&prog);
  }
  g_cache[key] = c;
  if (err) *err = c.err;
  return c.fn;
}

hipError_t codegen_launch(hipFunction_t fn, int dtype, const std::vector<const void*>& leaves,
                          void* out, int64_t n_total, hipStream_t s) {
  const int V = dtype == HEXLA_F32 ? 4 : 2;
  long n_pack = long(n_total / V);
  long total = long(n_total);
  std::vector<void*> args;
  std::vector<const void*> ptrs(leaves);
  for (size_t i = 0; i < ptrs.size(); ++i) args.push_back(&ptrs[i]);
  args.push_back(&out);
  args.push_back(&n_pack);
  args.push_back(&total);
  const long threads = n_pack + (n_total - n_pack * V);
  const long blocks = (threads + 255) / 256;
  if (blocks == 0) return hipSuccess;
  return hipModuleLaunchKernel(fn, unsigned(blocks), 1, 1, 256, 1, 1, 0, s, args.data(), nullptr);
}

}  // namespace hexla
