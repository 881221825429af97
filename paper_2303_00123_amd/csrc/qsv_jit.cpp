// Specialised tile-pass kernels.
//
// The tile kernel (qsv_tile.hip) interprets a pass record: per gate it loads
// an opcode, jumps through a switch of compile-time register bodies and
// writes its result into the other of two register sets.  The switch costs
// scalar instructions per gate, and the register sets cost moves (a
// controlled X becomes a copy of every amplitude).  Here a pass record is
// turned into the source of one kernel for that pass's structure: every
// gate is a direct call of its register body, updating the amplitudes in
// place, and every stage mapping, LDS offset and global offset is a
// constant.  The compiler then renames registers instead of moving them.
// Gate matrices are still read from the record in device memory, so a
// circuit with the same structure and new angles reuses the kernel.
//
// Kernels are compiled by the ROCm device compiler in child processes (the
// in-process runtime compiler serialises its compilations), several passes
// at once, then loaded with hipModuleLoadData.  A context keeps them, keyed
// by a hash of the record's structure (everything but the matrices).
#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "qsv_common.h"
#include "qsv_internal.h"

extern char** environ;

namespace qsv {

// Header texts the generated sources include (embedded at build time).
extern const char* const kJitFileNames[];
extern const char* const kJitFileTexts[];
extern const int kJitFileCount;

namespace {

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

template <typename R>
uint64_t record_key_t(const char* rec, bool split) {
    const TPassHdr* hd = reinterpret_cast<const TPassHdr*>(rec);
    const int ns = hd->nstages;
    uint64_t h = 1469598103934665603ull;
    const int32_t tag[3] = {int32_t(sizeof(R)), split ? 1 : 0, 2 /* generator version */};
    h = fnv1a(tag, sizeof(tag), h);
    if (const char* f = std::getenv("QSV_JIT_CFLAGS")) h = fnv1a(f, std::strlen(f), h);
    h = fnv1a(rec, sizeof(TPassHdr), h);
    h = fnv1a(rec + sizeof(TPassHdr), size_t(ns) * sizeof(TStage), h);
    const TGate<R>* g = reinterpret_cast<const TGate<R>*>(rec + sizeof(TPassHdr) + size_t(ns) * sizeof(TStage));
    for (int i = 0; i < hd->ngates; ++i) {
        const int32_t s4[4] = {g[i].kind, g[i].r0, g[i].r1, g[i].cs};
        h = fnv1a(s4, sizeof(s4), h);
    }
    return h;
}

// Expression for the LDS byte base of a thread: the swizzled half- or
// whole-tile index of the thread's bits, scaled by the amplitude size.  The
// swizzle is linear over GF(2), so it is the XOR of the swizzled images of
// the thread bits that are set.
std::string lds_base_expr(const int32_t* tbits, int nt, int esize) {
    std::ostringstream o;
    o << "(0u";
    for (int j = 0; j < nt; ++j) {
        const uint32_t img = tile_swz(1u << tbits[j], esize) * uint32_t(esize);
        o << " ^ ((0u - ((tid >> " << j << ") & 1u)) & 0x" << std::hex << img << std::dec << "u)";
    }
    o << ")";
    return o.str();
}

std::string deposit_expr(const int32_t* tpos, int nt) {
    std::ostringstream o;
    o << "(uint64_t(0)";
    for (int j = 0; j < nt; ++j) o << " | (uint64_t((tid >> " << j << ") & 1u) << " << tpos[j] << ")";
    o << ")";
    return o.str();
}

template <typename R>
std::string source_t(const char* rec, bool split, const std::string& fname) {
    using V = typename V2T<R>::type;
    const TPassHdr* hd = reinterpret_cast<const TPassHdr*>(rec);
    const TStage* st = reinterpret_cast<const TStage*>(rec + sizeof(TPassHdr));
    const int ns = hd->nstages, K = hd->k, RB = hd->rb, TB = K - RB, P = 1 << RB;
    const size_t goff = sizeof(TPassHdr) + size_t(ns) * sizeof(TStage);
    const TGate<R>* gt = reinterpret_cast<const TGate<R>*>(rec + goff);
    const int es = int(sizeof(V));
    const char* rt = sizeof(R) == 8 ? "double" : "float";
    std::ostringstream o;
    o << "#include \"qsv_tile_core.h\"\n"
      << "using namespace qsv;\nusing namespace qsv::tile;\n"
      << "extern \"C\" __global__ __launch_bounds__(" << (1 << TB) << ", 2) void " << fname
      << "(V2T<" << rt << ">::type* __restrict__ s, const char* __restrict__ plan, int from_zero) {\n"
      << "  using R = " << rt << ";\n  using V = V2T<R>::type;\n"
      << "  __shared__ V tile[" << (split ? (1 << (K - 1)) : (1 << K)) << "];\n"
      << "  char* const lds = reinterpret_cast<char*>(tile);\n"
      << "  const TGate<R>* __restrict__ G = reinterpret_cast<const TGate<R>*>(plan + " << goff << ");\n"
      << "  const uint32_t tid = threadIdx.x;\n"
      << "  const uint32_t ntiles = gridDim.x;\n"
      << "  uint64_t b = blockIdx.x;\n"
      << "  if ((ntiles & 7u) == 0) b = (blockIdx.x & 7u) * (ntiles >> 3) + (blockIdx.x >> 3);\n";
    for (int i = 0; i < K; ++i) o << "  b = insert0(b, " << hd->pos[i] << ");\n";
    o << "  const uint64_t xt = b | " << deposit_expr(hd->tpos_ld, TB) << ";\n"
      << "  V v[" << P << "];\n"
      << "  __builtin_amdgcn_s_setprio(2);\n"
      << "  if (from_zero) {\n";
    for (int u = 0; u < P; ++u)
        o << "    v[" << u << "].x = (xt | 0x" << std::hex << hd->du[u] << std::dec
          << "ull) == 0 ? R(1) : R(0); v[" << u << "].y = R(0);\n";
    o << "  } else {\n    const V* sp = s + xt;\n";
    for (int u = 0; u < P; ++u) o << "    v[" << u << "] = ld_nt(sp + 0x" << std::hex << hd->du[u] << std::dec << "ull);\n";
    o << "  }\n  __builtin_amdgcn_s_setprio(0);\n";
    auto gate_call = [&](int gi) {
        const TGate<R>& g = gt[gi];
        std::ostringstream c;
        const std::string m = "G[" + std::to_string(gi) + "].m";
        switch (g.kind) {
        case DK_1Q: c << "rg_1q<" << g.r0 << ">(v, v, " << m << ");"; break;
        case DK_1D: c << "rg_1d<" << g.r0 << ">(v, v, " << m << ");"; break;
        case DK_1R: c << "rg_1r<" << g.r0 << ">(v, v, " << m << ");"; break;
        case DK_C1Q: c << "rg_c1q<" << g.r0 << ", " << g.r1 << ">(v, v, " << m << ");"; break;
        case DK_CX: c << "rg_cx<" << g.r0 << ", " << g.r1 << ", true>(v, v);"; break;
        case DK_CD: c << "rg_cd<" << g.r0 << ", " << g.r1 << ">(v, v, " << m << ");"; break;
        case DK_2Q: c << "rg_2q<" << g.r0 << ", " << g.r1 << ">(v, v, " << m << ");"; break;
        default: return std::string();
        }
        return c.str();
    };
    for (int si = 0; si < ns; ++si) {
        const TStage& S = st[si];
        o << "  // stage " << si << "\n";
        if (!split && si > 0) {
            o << "  {\n    const uint32_t sb = " << lds_base_expr(S.tbits, TB, es) << ";\n";
            for (int u = 0; u < P; ++u)
                o << "    v[" << u << "] = *reinterpret_cast<const V*>(lds + (sb ^ 0x" << std::hex << S.su[u]
                  << std::dec << "u));\n";
            o << "  }\n";
        }
        for (int gi = S.gbeg; gi < S.gend; ++gi) {
            const std::string c = gate_call(gi);
            if (c.empty()) return std::string();
            o << "  " << c << "\n";
        }
        if (si + 1 >= ns) continue;
        if (!split) {
            o << "  {\n    const uint32_t sb = " << lds_base_expr(S.tbits, TB, es) << ";\n";
            for (int u = 0; u < P; ++u)
                o << "    *reinterpret_cast<V*>(lds + (sb ^ 0x" << std::hex << S.su_wr[u] << std::dec
                  << "u)) = v[" << u << "];\n";
            o << "    lds_barrier();\n  }\n";
            continue;
        }
        const TStage& N = st[si + 1];
        const int jw = S.jw;
        if (jw < 0 || jw >= RB) return std::string();
        o << "  {\n    const uint32_t sbw = " << lds_base_expr(S.tbw, TB, es) << ";\n"
          << "    const uint32_t sbr = " << lds_base_expr(N.tbr, TB, es) << ";\n"
          << "    V w[" << P / 2 << "];\n    __builtin_amdgcn_s_setprio(2);\n";
        if (si > 0) o << "    lds_barrier();\n";
        for (int rho = 0; rho < 2; ++rho) {
            for (int u = 0; u < P; ++u)
                if (((u >> jw) & 1) == rho)
                    o << "    *reinterpret_cast<V*>(lds + (sbw ^ 0x" << std::hex << S.su_wr[u] << std::dec
                      << "u)) = v[" << u << "];\n";
            o << "    lds_barrier();\n";
            for (int u = rho * P / 2; u < (rho + 1) * P / 2; ++u)
                o << "    " << (rho == 0 ? "w[" + std::to_string(u) + "]" : "v[" + std::to_string(u) + "]")
                  << " = *reinterpret_cast<const V*>(lds + (sbr ^ 0x" << std::hex << N.su[u] << std::dec
                  << "u));\n";
            if (rho == 0) o << "    lds_barrier();\n";
        }
        for (int u = 0; u < P / 2; ++u) o << "    v[" << u << "] = w[" << u << "];\n";
        o << "    __builtin_amdgcn_s_setprio(0);\n  }\n";
    }
    // the store address is formed anew (opaque to the compiler), so the
    // load addresses need not stay live across the whole pass
    o << "  uint64_t xs = b | " << deposit_expr(hd->tpos_st, TB) << ";\n"
      << "  asm volatile(\"\" : \"+v\"(xs));\n"
      << "  V* const sq = s + xs;\n"
      << "  __builtin_amdgcn_s_setprio(2);\n";
    for (int u = 0; u < P; ++u)
        o << "  st_nt(sq + 0x" << std::hex << hd->du_st[u] << std::dec << "ull, v[" << u << "]);\n";
    o << "}\n";
    return o.str();
}

std::string compiler_path() {
    if (const char* c = std::getenv("QSV_JIT_CLANG")) return c;
    std::string root = "/opt/rocm";
    if (const char* r = std::getenv("ROCM_PATH")) root = r;
    return root + "/llvm/bin/clang++";
}

bool write_file(const std::string& path, const std::string& text) {
    std::ofstream f(path, std::ios::binary);
    f << text;
    return bool(f);
}

bool read_file(const std::string& path, std::string& out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::ostringstream ss;
    ss << f.rdbuf();
    out = ss.str();
    return true;
}

// Resource usage of the compiled kernel from the compiler's remarks: true
// if it keeps two waves per SIMD and spills at most a few registers to
// scratch memory (QSV_JIT_MAX_SCRATCH bytes per lane, default 128: passes
// full of dense 2-qubit gates, whose 16 complex entries compete with the
// amplitudes for registers, spill a handful of values, and such a kernel
// still runs well ahead of the interpreting one).
bool resources_ok(const std::string& log) {
    auto field = [&](const char* key) {
        const size_t p = log.find(key);
        if (p == std::string::npos) return -1;
        return std::atoi(log.c_str() + p + std::strlen(key));
    };
    int max_scratch = 128;
    if (const char* m = std::getenv("QSV_JIT_MAX_SCRATCH")) max_scratch = std::atoi(m);
    const int scratch = field("ScratchSize [bytes/lane]: ");
    const int occ = field("Occupancy [waves/SIMD]: ");
    return scratch >= 0 && scratch <= max_scratch && occ >= 2;
}

struct Job {
    std::string dir, name, src, co, log;
    pid_t pid = -1;
    bool ok = false;
};

pid_t spawn_compile(const std::string& clang, Job& j) {
    std::vector<std::string> args = {clang, "-x", "hip", "--offload-arch=gfx950", "--cuda-device-only",
                                     "--no-gpu-bundle-output", "-O3", "-std=c++17", "-Xclang",
                                     "-target-feature", "-Xclang", "-packed-fp32-ops",
                                     "-Rpass-analysis=kernel-resource-usage", "-I", j.dir, j.src, "-o", j.co};
    // extra compiler options (QSV_JIT_CFLAGS, whitespace-separated), e.g. a
    // scheduling strategy to try
    if (const char* f = std::getenv("QSV_JIT_CFLAGS")) {
        std::istringstream in(f);
        for (std::string a; in >> a;) args.insert(args.end() - 2, a);
    }
    std::vector<char*> argv;
    for (auto& a : args) argv.push_back(const_cast<char*>(a.c_str()));
    argv.push_back(nullptr);
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addopen(&fa, 1, j.log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
    posix_spawn_file_actions_adddup2(&fa, 1, 2);
    pid_t pid = -1;
    if (posix_spawn(&pid, clang.c_str(), &fa, nullptr, argv.data(), environ) != 0) pid = -1;
    posix_spawn_file_actions_destroy(&fa);
    return pid;
}

}  // namespace

uint64_t jit_record_key(int dtype, const char* rec, bool split) {
    return dtype == QSV_C128 ? record_key_t<double>(rec, split) : record_key_t<float>(rec, split);
}

std::string jit_pass_source(int dtype, const char* rec, bool split, const std::string& fname) {
    return dtype == QSV_C128 ? source_t<double>(rec, split, fname) : source_t<float>(rec, split, fname);
}

bool jit_available() {
    struct stat sb;
    return stat(compiler_path().c_str(), &sb) == 0 && (sb.st_mode & S_IXUSR);
}

// Make sure every record in recs has a loaded kernel in ctx->jit; passes
// whose compilation fails or whose kernel would spill get a null entry (the
// caller runs the interpreting kernel for them).  Compiles run in child
// processes, up to `par` at once.
hipError_t jit_prepare(qsv_ctx ctx, int dtype, const std::vector<const char*>& recs,
                       const std::vector<bool>& split, std::vector<hipFunction_t>& fns) {
    fns.assign(recs.size(), nullptr);
    std::vector<uint64_t> keys(recs.size());
    std::vector<size_t> todo;
    for (size_t i = 0; i < recs.size(); ++i) {
        if (!recs[i]) continue;
        keys[i] = jit_record_key(dtype, recs[i], split[i]);
        auto it = ctx->jit_kernels.find(keys[i]);
        if (it != ctx->jit_kernels.end()) fns[i] = it->second.fn;
        else if (std::find_if(todo.begin(), todo.end(), [&](size_t t) { return keys[t] == keys[i]; }) == todo.end())
            todo.push_back(i);
    }
    if (todo.empty()) {
        for (size_t i = 0; i < recs.size(); ++i)
            if (recs[i] && !fns[i]) fns[i] = ctx->jit_kernels[keys[i]].fn;
        return hipSuccess;
    }
    const auto t0 = std::chrono::steady_clock::now();
    std::string base = "/tmp";
    if (const char* t = std::getenv("TMPDIR")) base = t;
    std::string tmpl = base + "/qsvjit-XXXXXX";
    std::vector<char> tb(tmpl.begin(), tmpl.end());
    tb.push_back('\0');
    if (!mkdtemp(tb.data())) return hipErrorUnknown;
    const std::string dir(tb.data());
    for (int f = 0; f < kJitFileCount; ++f) write_file(dir + "/" + kJitFileNames[f], kJitFileTexts[f]);
    std::vector<Job> jobs(todo.size());
    for (size_t k = 0; k < todo.size(); ++k) {
        Job& j = jobs[k];
        j.dir = dir;
        // one name per structure: traces aggregate the family by its prefix
        char hex[17];
        std::snprintf(hex, sizeof(hex), "%016llx", static_cast<unsigned long long>(keys[todo[k]]));
        j.name = std::string(dtype == QSV_C128 ? "qsv_pass_c128_" : "qsv_pass_c64_") + hex;
        j.src = dir + "/" + j.name + ".hip";
        j.co = dir + "/" + j.name + ".co";
        j.log = dir + "/" + j.name + ".log";
        const std::string text = jit_pass_source(dtype, recs[todo[k]], split[todo[k]], j.name);
        j.ok = !text.empty() && write_file(j.src, text);
    }
    // persistent cache of accepted kernels (QSV_JIT_CACHE names a directory)
    std::string cache;
    if (const char* c = std::getenv("QSV_JIT_CACHE")) cache = c;
    std::vector<std::string> cached_co(jobs.size());
    if (!cache.empty())
        for (size_t k = 0; k < jobs.size(); ++k) {
            const std::string path = cache + "/" + jobs[k].name + ".co";
            if (jobs[k].ok && read_file(path, cached_co[k]) && !cached_co[k].empty()) jobs[k].ok = false;
            else cached_co[k].clear();
        }
    const std::string clang = compiler_path();
    int par = int(std::thread::hardware_concurrency());
    if (const char* p = std::getenv("QSV_JIT_JOBS")) par = std::atoi(p);
    par = std::max(1, std::min(par, 16));
    size_t next = 0, running = 0;
    std::vector<size_t> live;
    while (next < jobs.size() || running > 0) {
        while (running < size_t(par) && next < jobs.size()) {
            Job& j = jobs[next];
            if (j.ok) {
                j.pid = spawn_compile(clang, j);
                if (j.pid > 0) ++running;
                else j.ok = false;
            }
            ++next;
        }
        if (running == 0) break;
        int status = 0;
        const pid_t pid = waitpid(-1, &status, 0);
        if (pid <= 0) break;
        for (Job& j : jobs)
            if (j.pid == pid) {
                j.pid = -1;
                --running;
                if (!WIFEXITED(status) || WEXITSTATUS(status) != 0) j.ok = false;
            }
    }
    hipError_t err = hipSuccess;
    int loaded = 0;
    for (size_t k = 0; k < jobs.size(); ++k) {
        Job& j = jobs[k];
        JitKernel jk{};
        std::string log, co;
        const bool from_cache = !cached_co[k].empty();
        if (from_cache) co.swap(cached_co[k]);
        if (from_cache || (j.ok && read_file(j.log, log) && resources_ok(log) && read_file(j.co, co))) {
            if (!from_cache && !cache.empty()) {
                mkdir(cache.c_str(), 0755);
                const std::string tmp = cache + "/" + j.name + ".co.tmp" + std::to_string(getpid());
                if (write_file(tmp, co)) std::rename(tmp.c_str(), (cache + "/" + j.name + ".co").c_str());
            }
            hipModule_t mod = nullptr;
            hipError_t e = hipModuleLoadData(&mod, co.data());
            if (e == hipSuccess) {
                hipFunction_t fn = nullptr;
                e = hipModuleGetFunction(&fn, mod, j.name.c_str());
                if (e == hipSuccess) {
                    jk.mod = mod;
                    jk.fn = fn;
                    ++loaded;
                } else {
                    (void)hipModuleUnload(mod);
                }
            }
            if (e != hipSuccess) err = e;
        } else {
            logf("jit: pass %zu not specialised (compile failed or kernel would spill)", k);
        }
        ctx->jit_kernels[keys[todo[k]]] = jk;   // null entries are remembered too
        std::remove(j.src.c_str());
        std::remove(j.co.c_str());
        std::remove(j.log.c_str());
    }
    for (int f = 0; f < kJitFileCount; ++f) std::remove((dir + "/" + kJitFileNames[f]).c_str());
    rmdir(dir.c_str());
    ctx->jit_compile_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ctx->jit_compiled += loaded;
    for (size_t i = 0; i < recs.size(); ++i)
        if (recs[i]) fns[i] = ctx->jit_kernels[keys[i]].fn;
    return err;
}

void jit_release(qsv_ctx ctx) {
    for (auto& kv : ctx->jit_kernels)
        if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
    ctx->jit_kernels.clear();
}

}  // namespace qsv
