// Pass kernels compiled at run time for one pass program each (see jit.hpp).
#include "jit.hpp"

#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <thread>

namespace sf {

// the text of sf_device.hpp and pass_dev.hpp, built into the library (jit_headers.cpp, written
// by the build from the sources)
extern const char *const kJitHeaderNames[2];
extern const char *const kJitHeaderText[2];

namespace {

std::string num(long long v) { return std::to_string(v); }

std::string hex64(uint64_t v)
{
    char b[32];
    std::snprintf(b, sizeof(b), "0x%016llxull", (unsigned long long)v);
    return b;
}

// One diagonal group as straight-line code: the lane part (mB, cmask, keep, pval) from its terms
// in the order the run-time evaluation reads them (pass_dev.hpp, apply_diag), then the register
// part with the group's flags, projected register bits and register weights as constants.
std::string diag_code(const DiagGroup &g, const std::vector<uint8_t> &terms)
{
    std::string s = "    {\n        int mB = 0;\n        uint32_t cmask = 0;\n        bool keep = true;\n"
                    "        uint32_t pval = 0;\n";
    size_t t = 2 * (size_t)g.term_off;
    auto a = [&](int i) { return num(terms[t + i]); };
    for (int i = 0; i < g.n_lin_b; ++i, t += 2)
        s += "        mB += " + a(1) + " * (int)((eB >> " + a(0) + ") & 1u);\n";
    for (int i = 0; i < g.n_quad_bb; ++i, t += 2)
        s += "        mB += 4 * (int)((eB >> " + a(0) + ") & (eB >> " + a(1) + ") & 1u);\n";
    for (int i = 0; i < g.n_quad_br; ++i, t += 2)
        s += "        cmask ^= ((uint32_t)(eB >> " + a(0) + ") & 1u) << " + a(1) + ";\n";
    for (int i = 0; i < g.n_zs_b; ++i, t += 2)
        s += "        mB += 4 * (int)((eB >> " + a(0) + ") & (sp >> " + a(1) + ") & 1u);\n";
    for (int i = 0; i < g.n_zs_r; ++i, t += 2)
        s += "        cmask ^= ((uint32_t)(sp >> " + a(1) + ") & 1u) << " + a(0) + ";\n";
    for (int i = 0; i < g.n_proj_b; ++i, t += 2)
        s += "        keep = keep && (((eB >> " + a(0) + ") & 1u) == ((sp >> " + a(1) + ") & 1u));\n";
    uint32_t pset = 0;
    for (int i = 0; i < g.n_proj_r; ++i, t += 2) {
        const int k = terms[t], u = terms[t + 1];
        if ((pset >> k) & 1u) {
            // a second projector on the same register qubit: zero unless both path bits agree
            s += "        keep = keep && ((uint32_t)((sp >> " + num(u) + ") & 1u) == ((pval >> " + num(k) + ") & 1u));\n";
        } else {
            s += "        pval |= (uint32_t)((sp >> " + num(u) + ") & 1u) << " + num(k) + ";\n";
            pset |= 1u << k;
        }
    }
    s += "        sf::diag_regs<R, T>(sf::CtGroup<" + num(g.flags) + "u, " + num(pset) + "u, " + hex64(g.tab[0]) + ", " +
         hex64(g.tab[1]) + ", " + hex64(g.tab[2]) + ", " + hex64(g.tab[3]) + ">{}, mB, cmask, keep, pval, v);\n    }\n";
    return s;
}

std::string prog_struct(const std::string &name, const std::string &body)
{
    return "struct " + name + " {\n    template <int R, typename T, typename C>\n"
           "    __device__ static __forceinline__ void apply(C (&v)[1 << R], const int lane, const uint64_t eB,\n"
           "                                                 const uint64_t sp)\n    {\n"
           "        (void)lane;\n        (void)eB;\n        (void)sp;\n" + body + "    }\n};\n";
}

std::mutex g_mu;                                               // cache and compiles
std::map<std::pair<int, std::string>, hipFunction_t> g_cache;  // (device, source) -> kernel

std::string kernel_name(const std::string &src)
{
    char b[40];
    std::snprintf(b, sizeof(b), "sfj_%016llx", (unsigned long long)std::hash<std::string>{}(src));
    return b;
}

std::string replace_all(std::string s, const std::string &from, const std::string &to)
{
    for (size_t p = s.find(from); p != std::string::npos; p = s.find(from, p + to.size())) s.replace(p, from.size(), to);
    return s;
}

// one hiprtc program: code object or error text
struct Unit {
    std::string src;
    std::vector<char> code;
    std::string err;
};

void compile_unit(Unit &u, const std::string &arch)
{
    hiprtcProgram prog;
    hiprtcResult r = hiprtcCreateProgram(&prog, u.src.c_str(), "sf_pass_jit.hip", 2, kJitHeaderText, kJitHeaderNames);
    if (r != HIPRTC_SUCCESS) {
        u.err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
        return;
    }
    const std::string off = "--offload-arch=" + arch;
    // the same code-generation options as the library's own kernels (packed FP32 off)
    const char *opts[] = {off.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        u.err = std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        hiprtcDestroyProgram(&prog);
        return;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    u.code.resize(n);
    hiprtcGetCode(prog, u.code.data());
    hiprtcDestroyProgram(&prog);
}

}  // namespace

std::string jit_program(const PassPlan &pp)
{
    if (pp.dense) return "";
    std::string body;
    for (const PassOp &op : pp.ops) {
        if (op.type == PO_REG) {
            body += "        sf::reg_gate<" + num(op.target) + ", R>(" + num(op.kind) + ", v);\n";
        } else if (op.type == PO_LANE) {
            body += "        sf::lane_gate<R>(" + num(op.target) + ", " + num(op.kind) + ", lane, v);\n";
        } else if (op.type == PO_DIAG) {
            if (op.group >= pp.groups.size()) return "";
            body += diag_code(pp.groups[op.group], pp.terms);
        } else if (op.type == PO_ISWAP) {
            // the same dispatch as the interpreted pass (pass_dev.hpp), with constant positions
            const std::string t0 = num(op.target), t1 = num(op.group & 0xffu);
            if (op.kind == 0) body += "        sf::reg_iswap_dispatch<R>(" + t0 + ", " + t1 + ", v);\n";
            else if (op.kind == 3) body += "        sf::lane_iswap<R>(" + t0 + ", " + t1 + ", lane, v);\n";
            else if (op.kind == 1) body += "        sf::reg_lane_iswap_dispatch<R>(" + t1 + ", " + t0 + ", lane, v);\n";
            else body += "        sf::reg_lane_iswap_dispatch<R>(" + t0 + ", " + t1 + ", lane, v);\n";
        } else if (op.type == PO_PFLIP_REG || op.type == PO_PFLIP_LANE) {
            // flip where path bits u and u + 1 differ, times i there for kind 1
            const std::string u = num(op.group), u1 = num(op.group + 1);
            body += "    {\n        const bool f = (((sp >> " + u + ") ^ (sp >> " + u1 + ")) & 1u) != 0;\n";
            if (op.type == PO_PFLIP_REG) body += "        sf::reg_flip_dispatch<R>(" + num(op.target) + ", f, v);\n";
            else body += "        sf::lane_flip<R>(" + num(op.target) + ", f, v);\n";
            if (op.kind)
                body += "#pragma unroll\n        for (int j = 0; j < (1 << R); ++j) {\n"
                        "            const T x = v[j].x, y = v[j].y;\n            v[j].x = f ? -y : x;\n"
                        "            v[j].y = f ? x : y;\n        }\n";
            body += "    }\n";
        } else {
            return "";
        }
    }
    return body;
}

std::string jit_kernel(bool fp64, int R0, const std::string &prog0, bool zskip0, int R1, const std::string &prog1,
                       bool zskip1)
{
    const std::string T = fp64 ? "double" : "float";
    auto body = [&](int R, bool z, const char *P, const char *a, const char *blk, const char *nblk) {
        return std::string("sf::pass_body<") + T + ", " + num(R) + ", false, " + (z ? "true" : "false") +
               ", sf::PassArgs, SFJ_NS::" + P + ">(" + a + ", " + blk + ", " + nblk + ");";
    };
    std::string s = "namespace SFJ_NS {\n" + prog_struct("P0", prog0);
    if (!prog1.empty()) s += prog_struct("P1", prog1);
    s += "}\n";
    const std::string head = "extern \"C\" __global__ __launch_bounds__(256) SF_PASS_OCCUPANCY void SFJ_KERNEL";
    if (prog1.empty()) {
        s += head + "(sf::PassArgs a)\n{\n    " + body(R0, zskip0, "P0", "a", "blockIdx.x", "gridDim.x") + "\n}\n";
    } else {
        s += head + "(sf::PassArgs a0, sf::PassArgs a1, uint32_t grid0)\n{\n    if (blockIdx.x < grid0) " +
             body(R0, zskip0, "P0", "a0", "blockIdx.x", "grid0") + "\n    else " +
             body(R1, zskip1, "P1", "a1", "blockIdx.x - grid0", "gridDim.x - grid0") + "\n}\n";
    }
    return s;
}

namespace {

// the sources as units of a few kernels each, their placeholders filled (kernel_name)
std::vector<Unit> make_units(const std::vector<std::string> &uniq, size_t n_threads,
                             std::vector<std::vector<size_t>> &members)
{
    const size_t per = (uniq.size() + n_threads - 1) / n_threads;
    std::vector<Unit> units;
    for (size_t b = 0; b < uniq.size(); b += per) {
        Unit u;
        u.src = "#include \"pass_dev.hpp\"\n";
        std::vector<size_t> m;
        for (size_t i = b; i < std::min(uniq.size(), b + per); ++i) {
            const std::string name = kernel_name(uniq[i]);
            u.src += replace_all(replace_all(uniq[i], "SFJ_NS", name + "_ns"), "SFJ_KERNEL", name);
            m.push_back(i);
        }
        units.push_back(std::move(u));
        members.push_back(std::move(m));
    }
    return units;
}

size_t compile_threads(size_t n)
{
    return std::max<size_t>(1, std::min<size_t>({16, n, (size_t)std::max(1u, std::thread::hardware_concurrency())}));
}

void compile_all(std::vector<Unit> &units, const std::string &arch)
{
    std::vector<std::thread> th;
    for (size_t i = 1; i < units.size(); ++i) th.emplace_back(compile_unit, std::ref(units[i]), std::cref(arch));
    if (!units.empty()) compile_unit(units[0], arch);
    for (std::thread &t : th) t.join();
}

}  // namespace

int jit_compile_only(const std::vector<std::string> &sources, const std::string &arch, uint64_t *code_bytes,
                     std::string &err)
{
    std::vector<std::vector<size_t>> members;
    std::vector<Unit> units = make_units(sources, compile_threads(sources.size()), members);
    compile_all(units, arch);
    uint64_t n = 0;
    for (const Unit &u : units) {
        if (!u.err.empty()) { err = "compiling a pass kernel: " + u.err; return SF_ERR_UNSUPPORTED; }
        n += u.code.size();
    }
    if (code_bytes) *code_bytes = n;
    return SF_OK;
}

int jit_kernels(const std::vector<std::string> &sources, std::vector<hipFunction_t> &fns, double *compile_ms,
                std::string &err, bool compile)
{
    fns.assign(sources.size(), nullptr);
    if (compile_ms) *compile_ms = 0;
    if (sources.empty()) return SF_OK;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(he); return SF_ERR_DEVICE; }
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<size_t> missing;
    std::vector<std::string> uniq;
    for (size_t i = 0; i < sources.size(); ++i) {
        auto it = g_cache.find({dev, sources[i]});
        if (it != g_cache.end()) fns[i] = it->second;
        else if (std::find(uniq.begin(), uniq.end(), sources[i]) == uniq.end()) uniq.push_back(sources[i]);
    }
    if (!uniq.empty() && compile) {
        hipDeviceProp_t prop;
        if ((he = hipGetDeviceProperties(&prop, dev)) != hipSuccess) {
            err = std::string("hipGetDeviceProperties: ") + hipGetErrorString(he);
            return SF_ERR_DEVICE;
        }
        std::string arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
        const auto t0 = std::chrono::steady_clock::now();
        // a few kernels per hiprtc program, the programs compiled on up to 16 threads
        std::vector<std::vector<size_t>> members;
        std::vector<Unit> units = make_units(uniq, compile_threads(uniq.size()), members);
        compile_all(units, arch);
        for (const Unit &u : units)
            if (!u.err.empty()) { err = "compiling a pass kernel: " + u.err; return SF_ERR_DEVICE; }
        for (size_t ui = 0; ui < units.size(); ++ui) {
            hipModule_t mod;   // kept loaded until the process ends (its kernels stay in the cache)
            if ((he = hipModuleLoadData(&mod, units[ui].code.data())) != hipSuccess) {
                err = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
                return SF_ERR_DEVICE;
            }
            for (size_t i : members[ui]) {
                hipFunction_t fn;
                if ((he = hipModuleGetFunction(&fn, mod, kernel_name(uniq[i]).c_str())) != hipSuccess) {
                    err = std::string("hipModuleGetFunction: ") + hipGetErrorString(he);
                    return SF_ERR_DEVICE;
                }
                g_cache[{dev, uniq[i]}] = fn;
            }
        }
        if (compile_ms)
            *compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (size_t i = 0; i < sources.size(); ++i) fns[i] = g_cache[{dev, sources[i]}];
    }
    return SF_OK;
}

}  // namespace sf
