// Per-robot code generation and compilation (paper Sec. IV-C: the robot's topology is
// known when code is generated, so offsets, parents, level structure and zero patterns
// become constants of the kernel instead of run-time lookups).
//
// A topology (parent array) is turned into a prelude of compile-time tables and
// prepended to the hand-written device source; hiprtc compiles the result for gfx950.
// Code objects are cached on disk under a hash of the full source and options.
#include "grid_internal.h"

#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

namespace grid_impl {

// embedded copy of grid_device.hip (generated at build time)
#include "grid_device_src.inc"

bool analyse_topology(const int32_t* parent, int32_t n, Topology* out, std::string* err)
{
    if (n < 1 || n > kMaxBodies) {
        *err = "n must be in 1.." + std::to_string(kMaxBodies);
        return false;
    }
    Topology t;
    t.n = n;
    t.parent.assign(parent, parent + n);
    t.level.assign(n, 0);
    t.branch.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const int p = parent[i];
        if (p < -1 || p >= i) {
            *err = "parent[" + std::to_string(i) + "] = " + std::to_string(p) +
                   " must satisfy -1 <= parent[i] < i";
            return false;
        }
        t.level[i] = p < 0 ? 0 : t.level[p] + 1;
        t.branch[i] = p < 0 ? i : t.branch[p];
    }
    t.nlev = 0;
    for (int i = 0; i < n; ++i)
        t.nlev = std::max(t.nlev, t.level[i] + 1);
    t.level_mask.assign(t.nlev, 0);
    for (int i = 0; i < n; ++i)
        t.level_mask[t.level[i]] |= 1ull << i;
    // inward rounds, deepest level first: round k of a level holds the k-th child of every
    // parent, so no two bodies of a round add into the same parent
    t.round_mask.clear();
    for (int l = t.nlev - 1; l >= 1; --l) {
        std::vector<std::vector<int>> kids(n);
        size_t rounds = 0;
        for (int i = 0; i < n; ++i)
            if (t.level[i] == l) {
                kids[parent[i]].push_back(i);
                rounds = std::max(rounds, kids[parent[i]].size());
            }
        for (size_t k = 0; k < rounds; ++k) {
            uint64_t m = 0;
            for (int p = 0; p < n; ++p)
                if (k < kids[p].size())
                    m |= 1ull << kids[p][k];
            t.round_mask.push_back(m);
        }
    }
    // related[i]: bodies on the same root path as i (ancestors, descendants, itself);
    // M_ik is structurally zero for every other k
    t.related.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        t.related[i] |= 1ull << i;
        for (int a = parent[i]; a >= 0; a = parent[a]) {
            t.related[i] |= 1ull << a;
            t.related[a] |= 1ull << i;
        }
    }
    t.max_anc = t.nlev - 1;
    int lanes = 2;
    while (lanes < 2 * n)
        lanes *= 2;
    t.lanes = lanes;
    *out = std::move(t);
    return true;
}

static void emit_int_array(std::ostringstream& os, const char* name, const std::vector<int>& v)
{
    os << "__device__ constexpr int " << name << "[" << std::max<size_t>(1, v.size()) << "] = {";
    if (v.empty())
        os << "0";
    for (size_t i = 0; i < v.size(); ++i)
        os << (i ? ", " : "") << v[i];
    os << "};\n";
}

static void emit_mask_array(std::ostringstream& os, const char* name,
                            const std::vector<uint64_t>& v)
{
    os << "__device__ constexpr unsigned long long " << name << "["
       << std::max<size_t>(1, v.size()) << "] = {";
    if (v.empty())
        os << "0ull";
    for (size_t i = 0; i < v.size(); ++i)
        os << (i ? ", " : "") << "0x" << std::hex << v[i] << std::dec << "ull";
    os << "};\n";
}

std::string generate_source(const Topology& t, uint32_t flags)
{
    std::ostringstream os;
    os << "// generated: one robot topology as compile-time tables\n";
    os << "#define GRID_N " << t.n << "\n";
    os << "#define GRID_L " << t.lanes << "\n";
    os << "#define GRID_NLEV " << t.nlev << "\n";
    os << "#define GRID_NROUND " << t.round_mask.size() << "\n";
    os << "#define GRID_MAXANC " << t.max_anc << "\n";
    os << "#define GRID_DYN_DOUBLE " << ((flags & GRID_FLAG_FP32_DYNAMICS) ? 0 : 1) << "\n";
    emit_int_array(os, "kParent", t.parent);
    emit_int_array(os, "kBranch", t.branch);
    emit_mask_array(os, "kRelated", t.related);
    emit_mask_array(os, "kLevelMask", t.level_mask);
    emit_mask_array(os, "kRoundMask", t.round_mask);
    os << "#line 1 \"grid_device.hip\"\n";
    os << grid_device_src;
    return os.str();
}

static const char* const kCompileOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17",
    // packed FP32 instructions are not generated (correctness of some packed forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

static uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_dir()
{
    if (const char* env = std::getenv("GRID_KERNEL_CACHE"))
        if (*env)
            return env;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&cache_dir), &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        size_t slash = so.rfind('/');
        std::string dir = slash == std::string::npos ? "." : so.substr(0, slash);
        return dir + "/_kcache";
    }
    return "/tmp/grid_kcache";
}

static bool read_file(const std::string& path, std::vector<char>* out)
{
    std::ifstream f(path, std::ios::binary);
    if (!f)
        return false;
    out->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return !out->empty();
}

static void write_file_atomic(const std::string& dir, const std::string& path,
                              const std::vector<char>& data)
{
    mkdir(dir.c_str(), 0755);
    std::string tmp = path + ".tmp" + std::to_string(getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f)
            return;   // cache is best effort
        f.write(data.data(), data.size());
        if (!f)
            return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

static std::mutex g_compile_mutex;

grid_status compile_cached(const std::string& source, std::vector<char>* code, std::string* err)
{
    std::string key_src = source;
    for (const char* o : kCompileOptions)
        key_src += std::string("\n//opt ") + o;
    char name[64];
    std::snprintf(name, sizeof name, "grid_%016llx.hsaco", (unsigned long long)fnv1a(key_src));
    const std::string dir = cache_dir();
    const std::string path = dir + "/" + name;
    if (read_file(path, code))
        return GRID_OK;

    std::lock_guard<std::mutex> lock(g_compile_mutex);
    if (read_file(path, code))
        return GRID_OK;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, source.c_str(), "grid_robot.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return GRID_ECOMPILE;
    }
    const int nopt = sizeof(kCompileOptions) / sizeof(kCompileOptions[0]);
    hiprtcResult rc = hiprtcCompileProgram(prog, nopt, kCompileOptions);
    if (rc != HIPRTC_SUCCESS) {
        size_t log_size = 0;
        hiprtcGetProgramLogSize(prog, &log_size);
        std::string log(log_size, '\0');
        if (log_size)
            hiprtcGetProgramLog(prog, &log[0]);
        *err = std::string("kernel compilation failed: ") + hiprtcGetErrorString(rc) + "\n" + log;
        hiprtcDestroyProgram(&prog);
        return GRID_ECOMPILE;
    }
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    code->resize(size);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    write_file_atomic(dir, path, *code);
    return GRID_OK;
}

}  // namespace grid_impl
