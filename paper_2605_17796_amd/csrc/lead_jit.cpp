// Run-time compilation of the specialised kernels (see lead_jit.hpp), with a
// cache of code objects on disk.
#include "lead_jit.hpp"
#include "lead_args.hpp"

#include <dlfcn.h>
#include <hip/hiprtc.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <utility>

namespace lead {
namespace jit {

// Texts of lead_args.hpp, lead_device.hpp and lead_spec.hpp, embedded at
// build time (the run-time compiler reads headers from memory).
extern const int kNumHeaders;
extern const char *const kHeaderNames[];
extern const char *const kHeaderTexts[];

namespace {

// hipRTC, opened on first use: the process may already hold a copy (the one
// PyTorch ships), which dlopen then returns.
struct Rtc {
    bool ok = false;
    std::string err;
    hiprtcResult (*create)(hiprtcProgram *, const char *, const char *, int, const char *const *,
                           const char *const *) = nullptr;
    hiprtcResult (*compile)(hiprtcProgram, int, const char *const *) = nullptr;
    hiprtcResult (*log_size)(hiprtcProgram, size_t *) = nullptr;
    hiprtcResult (*log)(hiprtcProgram, char *) = nullptr;
    hiprtcResult (*code_size)(hiprtcProgram, size_t *) = nullptr;
    hiprtcResult (*code)(hiprtcProgram, char *) = nullptr;
    hiprtcResult (*destroy)(hiprtcProgram *) = nullptr;
    hiprtcResult (*version)(int *, int *) = nullptr;   // optional
};

const Rtc &rtc() {
    static Rtc r;
    static std::once_flag once;
    std::call_once(once, [] {
        void *h = nullptr;
        for (const char *name : {"libhiprtc.so.7", "libhiprtc.so", "/opt/rocm/lib/libhiprtc.so.7"})
            if ((h = dlopen(name, RTLD_NOW | RTLD_LOCAL))) break;
        if (!h) {
            r.err = "hipRTC not found";
            return;
        }
        auto sym = [&](auto &fp, const char *s) {
            fp = reinterpret_cast<std::remove_reference_t<decltype(fp)>>(dlsym(h, s));
            return fp != nullptr;
        };
        r.ok = sym(r.create, "hiprtcCreateProgram") && sym(r.compile, "hiprtcCompileProgram") &&
               sym(r.log_size, "hiprtcGetProgramLogSize") && sym(r.log, "hiprtcGetProgramLog") &&
               sym(r.code_size, "hiprtcGetCodeSize") && sym(r.code, "hiprtcGetCode") &&
               sym(r.destroy, "hiprtcDestroyProgram");
        if (!r.ok) r.err = "hipRTC lacks an entry point";
        sym(r.version, "hiprtcVersion");
    });
    return r;
}

std::mutex g_mu;
std::map<std::string, std::vector<char>> g_objects;
std::map<std::pair<int, std::string>, std::shared_ptr<const Kernels>> g_modules;

int workgroup_for(int order) { return ((order + 63) / 64) * 64; }

// Whether the per-shot kernel's LDS (partner-exchange buffer D2 x wg and
// lambda' of the positions with sigma[j] >= j, wg each, f32) stays within
// 128 KB, leaving room for the per-shot flags and e_hat bitmaps.
bool lam_lds_fits(const Code &c, int t) {
    const int D2 = c.delta * c.delta, wg = workgroup_for(c.order);
    int no = 0;
    for (int j = 0; j < D2 && j < (int)c.t[t].sigma.size(); ++j) no += c.t[t].sigma[j] >= j ? 1 : 0;
    return (size_t)(D2 + no) * wg * sizeof(float) <= 128u * 1024u;
}

// Degree from which a check keeps the compressed state in the per-shot
// min-sum kernel (0: none): for views above kTwoWaveMaxEdges edges, the
// largest threshold that leaves at most kHybridExplicitEdges messages (those
// of the lower-degree checks) in registers.
int hybrid_degree(const TypeTables &tt) {
    if (tt.eloc <= kTwoWaveMaxEdges) return 0;
    int best = 1;   // every check compressed
    for (int i = 0; i < tt.r; ++i) {
        const int t = __builtin_popcountll(tt.mask[i]) + 1;
        int ex = 0;
        for (int k = 0; k < tt.r; ++k) {
            const int d = __builtin_popcountll(tt.mask[k]);
            if (d < t) ex += d;
        }
        if (ex <= kHybridExplicitEdges && t > best) best = t;
    }
    return best;
}

// ---- code objects on disk --------------------------------------------------
// A compiled code object is kept in a file named by a 128-bit hash of its key
// (compiler options, hipRTC version, the embedded headers and the generated
// source, which holds the code's check masks and position map).  The file
// stores the key itself, and a hit requires it to match byte for byte, so a
// hash collision can only cost a recompilation.  Directory: $LEAD_JIT_CACHE
// ("off" disables the cache), else _build/jit beside liblead.so.  Files are
// written to a temporary name and renamed, so concurrent processes never see
// a partial object.

const char *const kCompileOpts[] = {"--gpu-architecture=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                                    "-Xclang", "-packed-fp32-ops"};
constexpr int kNumCompileOpts = (int)(sizeof(kCompileOpts) / sizeof(kCompileOpts[0]));
constexpr char kCacheMagic[8] = {'L', 'E', 'A', 'D', 'C', 'O', '0', '1'};

std::string cache_key(const std::string &src) {
    std::string k;
    for (int i = 0; i < kNumCompileOpts; ++i) (k += kCompileOpts[i]) += '\n';
    int ma = 0, mi = 0;
    const Rtc &r = rtc();
    if (r.ok && r.version) r.version(&ma, &mi);
    k += "hiprtc " + std::to_string(ma) + "." + std::to_string(mi) + "\n";
    // the library file itself: builds of one version number (the system's
    // and one bundled with another package that loaded first) generate
    // different code
    Dl_info info{};
    struct stat st {};
    if (r.ok && dladdr(reinterpret_cast<void *>(r.create), &info) && info.dli_fname &&
        stat(info.dli_fname, &st) == 0)
        k += std::string(info.dli_fname) + " " + std::to_string((long long)st.st_size) + " " +
             std::to_string((long long)st.st_mtime) + "\n";
    for (int i = 0; i < kNumHeaders; ++i) {
        k += kHeaderNames[i];
        k += '\0';
        k += kHeaderTexts[i];
        k += '\0';
    }
    return k + src;
}

// FNV-1a, 64 bits, from two offset bases: a 128-bit file name.
std::string key_hash(const std::string &key) {
    uint64_t h[2] = {0xcbf29ce484222325ull, 0x6c62272e07bb0142ull};
    for (unsigned char ch : key)
        for (uint64_t &x : h) x = (x ^ ch) * 0x100000001b3ull;
    char buf[40];
    std::snprintf(buf, sizeof buf, "%016llx%016llx", (unsigned long long)h[0], (unsigned long long)h[1]);
    return buf;
}

const std::string &cache_dir() {
    static const std::string dir = [] {
        if (const char *e = std::getenv("LEAD_JIT_CACHE")) return std::string(std::strcmp(e, "off") ? e : "");
        Dl_info info{};
        if (!dladdr(reinterpret_cast<void *>(&cache_key), &info) || !info.dli_fname) return std::string();
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/_build/jit";
    }();
    return dir;
}

bool cache_read(const std::string &key, std::vector<char> &obj) {
    const std::string &dir = cache_dir();
    if (dir.empty()) return false;
    std::ifstream f(dir + "/lead_spec_" + key_hash(key) + ".co", std::ios::binary);
    if (!f) return false;
    char magic[8];
    uint64_t klen = 0, olen = 0;
    if (!f.read(magic, 8) || std::memcmp(magic, kCacheMagic, 8) || !f.read(reinterpret_cast<char *>(&klen), 8) ||
        klen != key.size())
        return false;
    std::string stored(klen, '\0');
    if (!f.read(&stored[0], (std::streamsize)klen) || stored != key) return false;
    if (!f.read(reinterpret_cast<char *>(&olen), 8) || olen == 0 || olen > (1ull << 30)) return false;
    obj.assign(olen, 0);
    return (bool)f.read(obj.data(), (std::streamsize)olen);
}

void cache_write(const std::string &key, const std::vector<char> &obj) {
    const std::string &dir = cache_dir();
    if (dir.empty()) return;
    // create the directory and its parent (_build) if missing
    const size_t slash = dir.rfind('/');
    if (slash != std::string::npos && slash > 0) mkdir(dir.substr(0, slash).c_str(), 0755);
    mkdir(dir.c_str(), 0755);
    const std::string path = dir + "/lead_spec_" + key_hash(key) + ".co";
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        const uint64_t klen = key.size(), olen = obj.size();
        f.write(kCacheMagic, 8);
        f.write(reinterpret_cast<const char *>(&klen), 8);
        f.write(key.data(), (std::streamsize)klen);
        f.write(reinterpret_cast<const char *>(&olen), 8);
        f.write(obj.data(), (std::streamsize)olen);
        if (!f) {
            f.close();
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

// LEAD_JIT_DUMP=<dir>: keep a copy of every code object this process
// compiles or reads from the cache, with its source (for inspection).
void dump(const std::string &src, const std::vector<char> &obj) {
    const char *dir = std::getenv("LEAD_JIT_DUMP");
    if (!dir) return;
    std::ostringstream name;
    name << dir << "/lead_spec_" << std::hex << std::hash<std::string>{}(src) << ".co";
    std::ofstream(name.str(), std::ios::binary).write(obj.data(), (std::streamsize)obj.size());
    std::ofstream(name.str() + ".hip") << src;
}

}  // namespace

bool osd_fits(const Code &c, int t) {
    const int m = c.order * c.t[t].r, W = (c.n + 63) / 64, RPL = (m + 255) / 256;
    return m > 0 && c.n > 0 && RPL * W <= kOsdMaxWords && RPL <= 32;
}

namespace {
// The lowest-degree checks (ties: lowest index) whose messages go to LDS
// until at most reg_max stay in registers, and their edges.
uint32_t lds_mask_for(const TypeTables &tt, int reg_max) {
    std::vector<int> order(tt.r);
    for (int i = 0; i < tt.r; ++i) order[i] = i;
    auto deg = [&](int i) { return __builtin_popcountll(tt.mask[i]); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg(x) < deg(y); });
    uint32_t m = 0u;
    int reg = tt.eloc;
    for (int i : order) {
        if (reg <= reg_max) break;
        m |= 1u << i;
        reg -= deg(i);
    }
    return m;
}
int mask_edges(const TypeTables &tt, uint32_t m) {
    int e = 0;
    for (int i = 0; i < tt.r; ++i)
        if ((m >> i) & 1u) e += __builtin_popcountll(tt.mask[i]);
    return e;
}
}  // namespace

bool local_alt(const TypeTables &tt) {
    if (tt.r > 32) return tt.eloc <= kTwoWaveMaxEdges;
    if (tt.eloc <= kTwoWaveMaxEdges) return true;
    return 64 * 4 * mask_edges(tt, lds_mask_for(tt, kLocalAltRegEdges)) <= kLocalAltLdsBytes;
}

uint32_t local_lds_mask(const TypeTables &tt) {
    if (tt.eloc <= kTwoWaveMaxEdges || tt.r > 32) return 0u;
    return lds_mask_for(tt, local_alt(tt) ? kLocalAltRegEdges : kLocalRegEdges);
}

int local_lds_edges(const TypeTables &tt) { return mask_edges(tt, local_lds_mask(tt)); }

bool tile_fits(const Code &c, int t) {
    const int D2 = c.delta * c.delta;
    if (c.order <= 64 || lead::kTileWG / c.order < 2 || (int)c.t[t].sigma.size() != D2) return false;
    // a slot's e_hat bitmap and words live at its lane offset
    if ((c.n + 31) / 32 > c.order || c.order < 16) return false;
    return tile_lds_bytes(c, t) <= 160u * 1024u;
}

size_t tile_lds_bytes(const Code &c, int t) {
    const int D2 = c.delta * c.delta;
    const std::vector<int> &sg = c.t[t].sigma;
    int na = 0, nb = 0, no = 0;
    for (int j = 0; j < D2 && j < (int)sg.size(); ++j) {
        na += sg[j] <= j ? 1 : 0;
        nb += sg[j] > j ? 1 : 0;
        no += sg[j] >= j ? 1 : 0;
    }
    const size_t rows = (size_t)std::max(na, nb) + no;   // exchange and lambda' rows
    const size_t npw = (size_t)(D2 + 15) / 16 * 4;       // partner-table words per view
    // rows, the slots' words (16 beyond the workgroup), four control words,
    // the e_hat bitmaps, the partner tables
    return rows * lead::kTileWG * 4 + (size_t)(lead::kTileWG + 16) * 4 + 4 * 4 + (size_t)lead::kTileWG * 4 +
           (size_t)c.order * npw * 4;
}

int osd_workgroup(const Code &c, int t) {
    const int m = c.order * c.t[t].r, RPL = (m + 255) / 256;
    return 64 * ((m + 64 * RPL - 1) / (64 * RPL));
}

bool osd_big_fits(const Code &c, int t) {
    const int m = c.order * c.t[t].r;
    return m > 0 && c.n > 0 && m <= kOsdBigMaxRows && c.n <= 65535;
}

int osd_big_workgroup(const Code &c, int t) {
    const int m = c.order * c.t[t].r;
    return std::min(512, 64 * ((m + 63) / 64));
}

size_t osd_big_slot_bytes(const Code &c, int t) {
    const size_t m = (size_t)c.order * c.t[t].r;
    return sizeof(uint64_t) * ((size_t)(c.n + 63) / 64 + 1) * m;
}

namespace {

// The compile-time description of check type t of code c (check masks,
// position map, edge tables) as a struct named `name`.
void emit_code_struct(std::ostringstream &o, const Code &c, int t, const std::string &name) {
    const TypeTables &tt = c.t[t];
    const int D = c.delta, D2 = D * D;
    int nfix = 0;
    for (int j = 0; j < D2; ++j) nfix += tt.sigma[j] == j;
    o << "struct " << name << " {\n"
      << "    static constexpr int D = " << D << ", R = " << tt.r << ", NFIX = " << nfix << ";\n"
      << "    static constexpr bool SPLIT = " << (tt.eloc > kTwoWaveMaxEdges ? "true" : "false") << ";\n"

      << "    static constexpr int HYB = " << hybrid_degree(tt) << ";\n"
      << "    static constexpr unsigned LDSMASK = " << local_lds_mask(tt) << "u;\n"
      << "    static constexpr bool LOCAL_ALT = " << (local_alt(tt) ? "true" : "false") << ";\n"
      << "    static constexpr bool LAM_LDS = " << (lam_lds_fits(c, t) ? "true" : "false") << ";\n"
      << "    static constexpr uint64_t mask[" << tt.r << "] = {";
    for (int i = 0; i < tt.r; ++i) o << (i ? ", " : "") << "0x" << std::hex << tt.mask[i] << std::dec << "ull";
    o << "};\n    static constexpr int sigma[" << D2 << "] = {";
    for (int j = 0; j < D2; ++j) o << (j ? ", " : "") << tt.sigma[j];
    o << "};\n";
    // edge tables
    std::ostringstream deg, base;
    int e = 0;
    for (int i = 0; i < tt.r; ++i) {
        const int k = __builtin_popcountll(tt.mask[i]);
        deg << (i ? ", " : "") << k;
        base << (i ? ", " : "") << e;
        e += k;
    }
    o << "    static constexpr int E = " << e << ";\n"
      << "    static constexpr int deg[" << tt.r << "] = {" << deg.str() << "};\n"
      << "    static constexpr int base[" << tt.r << "] = {" << base.str() << "};\n};\n";
}

}  // namespace

std::string source(const Code &c, int t, bool sp) {
    const TypeTables &tt = c.t[t];
    const int D = c.delta, D2 = D * D;
    if (tt.sigma.empty() || (int)tt.sigma.size() != D2) return std::string();
    if (sp && tt.eloc > kSumProductMaxEdges) return std::string();
    const int wg = workgroup_for(c.order);
    std::ostringstream o;
    o << "#include \"lead_spec.hpp\"\n";
    emit_code_struct(o, c, t, "LeadCode");
    for (int form = kCompressed; form <= kSumProduct; ++form) {
        if ((form == kSumProduct) != sp) continue;
        if (form != kCompressed && tt.eloc > kExplicitMaxEdges) continue;
        for (int pm = 0; pm < 2; ++pm)
            // min-sum with one prior per shot: three waves per SIMD (168
            // VGPRs) where a view's messages and sums fit them, at most
            // kThreeWaveMaxState registers (the queue kernel's loads in its
            // refill step need the third wave; with a prior per qubit the
            // priors would not fit; the 77-edge A5 X-check views spill at
            // three waves and run two)
            o << "extern \"C\" __global__ void __launch_bounds__(64"
              << (form != kSumProduct && pm == 0 &&
                          (form == kCompressed ? 4 * tt.r : tt.eloc) + D2 <= kThreeWaveMaxState
                      ? ", 3"
                      : (form == kExplicit && pm == 0 && local_lds_mask(tt) != 0u ? ", 2" : ""))
              << ") lead_spec_local_" << form << pm
              << "(lead::DecodeArgs a, lead::LocalArgs w) { lead_spec::local_body<LeadCode, " << pm << ", " << form
              << ">(a, w); }\n";
        // at least two waves per SIMD for the per-shot kernel (its rounds
        // wait on the partner exchange, which a lone wave cannot hide); the
        // compressed form within one wave keeps the whole register file, and
        // so does sum-product on views above kTwoWaveMaxEdges edges (one
        // register per message and no compressed alternative)
        const bool whole_file = (form == kCompressed && wg == 64) || (form == kSumProduct && tt.eloc > kTwoWaveMaxEdges);
        o << "extern \"C\" __global__ void __launch_bounds__(" << wg
          << (whole_file ? "" : ", 2")
          << ") lead_spec_global_" << form
          << "(lead::DecodeArgs a, lead::LocalArgs w, lead::SpecArgs x) { lead_spec::global_body<LeadCode, " << wg
          << ", " << (wg == 64 ? "true" : "false") << ", " << form << ">(a, w, x); }\n";
        // the persistent form for views spanning several waves
        if (form != kSumProduct && tile_fits(c, t))
            o << "extern \"C\" __global__ void __launch_bounds__(" << lead::kTileWG << ") lead_spec_tile_" << form
              << "(lead::DecodeArgs a, lead::LocalArgs w, lead::SpecArgs x) { lead_spec::global_tile_body<LeadCode, "
              << form << ">(a, w, x); }\n";
        // the explicit and sum-product forms without the fixed-point test of
        // global BP: the decode's Phases 2-3 kernel when that test is off
        if (form == kExplicit || form == kSumProduct) {
            if (form == kExplicit && tile_fits(c, t))
                o << "extern \"C\" __global__ void __launch_bounds__(" << lead::kTileWG << ") lead_spec_tile_" << form
                  << "n(lead::DecodeArgs a, lead::LocalArgs w, lead::SpecArgs x) { "
                     "lead_spec::global_tile_body<LeadCode, " << form << ", false>(a, w, x); }\n";
            else
                o << "extern \"C\" __global__ void __launch_bounds__(" << wg << (whole_file ? "" : ", 2")
                  << ") lead_spec_global_" << form
                  << "n(lead::DecodeArgs a, lead::LocalArgs w, lead::SpecArgs x) { lead_spec::global_body<LeadCode, "
                  << wg << ", " << (wg == 64 ? "true" : "false") << ", " << form << ", false, false>(a, w, x); }\n";
        }
        // the plain per-round form of the same kernel
        o << "extern \"C\" __global__ void __launch_bounds__(" << wg
          << (whole_file ? "" : ", 2")
          << ") lead_spec_round_" << form
          << "(lead::DecodeArgs a, lead::LocalArgs w, lead::SpecArgs x, lead::PlainArgs pl) { "
             "lead_spec::global_body<LeadCode, " << wg
          << ", " << (wg == 64 ? "true" : "false") << ", " << form << ", true>(a, w, x, pl); }\n";
    }
    o << "extern \"C\" __global__ void __launch_bounds__(64) lead_spec_local_osd(lead::DecodeArgs a, lead::LocalArgs w) "
         "{ lead_spec::local_osd_body<LeadCode>(a, w); }\n";
    if (osd_fits(c, t)) {
        const int m = c.order * tt.r;
        int sortn = 1;
        while (sortn < c.n) sortn <<= 1;
        const int owg = osd_workgroup(c, t);
        o << "struct LeadGlobal {\n    static constexpr int M = " << m << ", NQ = " << c.n << ", W = " << (c.n + 63) / 64
          << ", RPL = " << (m + 255) / 256 << ", WG = " << owg << ", RANK = " << tt.rank << ", SORTN = " << sortn
          << ";\n};\n"
          << "extern \"C\" __global__ void __launch_bounds__(" << owg
          << ") lead_spec_osd(lead::DecodeArgs a, lead::OsdArgs o) { lead_spec::osd_global_body<LeadGlobal, false>(a, o); }\n"
          << "extern \"C\" __global__ void __launch_bounds__(" << owg
          << ") lead_spec_osd_cs(lead::DecodeArgs a, lead::OsdArgs o) { lead_spec::osd_global_body<LeadGlobal, true>(a, o); }\n";
    }
    if (osd_big_fits(c, t)) {
        const int m = c.order * tt.r, bwg = osd_big_workgroup(c, t);
        int sortn = 1;
        while (sortn < c.n) sortn <<= 1;
        const int kc = std::max(1, std::min(4, sortn / 2048));
        o << "struct LeadGlobalBig {\n    static constexpr int M = " << m << ", NQ = " << c.n << ", W = " << (c.n + 63) / 64
          << ", RPL = " << (m + bwg - 1) / bwg << ", WG = " << bwg << ", RANK = " << tt.rank << ", SORTN = " << sortn
          << ", KC = " << kc << ";\n};\n"
          << "extern \"C\" __global__ void __launch_bounds__(" << bwg
          << ") lead_spec_osd_big(lead::DecodeArgs a, lead::OsdArgs o, lead::OsdBigArgs b) "
             "{ lead_spec::osd_big_body<LeadGlobalBig, false>(a, o, b); }\n"
          << "extern \"C\" __global__ void __launch_bounds__(" << bwg
          << ") lead_spec_osd_big_cs(lead::DecodeArgs a, lead::OsdArgs o, lead::OsdBigArgs b) "
             "{ lead_spec::osd_big_body<LeadGlobalBig, true>(a, o, b); }\n";
    }
    return o.str();
}

bool compile(const std::string &src, std::vector<char> &obj, std::string &err) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_objects.find(src);
        if (it != g_objects.end()) {
            obj = it->second;
            return true;
        }
    }
    const std::string key = cache_key(src);
    if (cache_read(key, obj)) {
        dump(src, obj);
        std::lock_guard<std::mutex> lk(g_mu);
        g_objects.emplace(src, obj);
        return true;
    }
    const Rtc &r = rtc();
    if (!r.ok) {
        err = r.err;
        return false;
    }
    hiprtcProgram prog = nullptr;
    if (r.create(&prog, src.c_str(), "lead_spec_code.hip", kNumHeaders, kHeaderTexts, kHeaderNames) !=
        HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    const hiprtcResult cr = r.compile(prog, kNumCompileOpts, kCompileOpts);
    bool ok = cr == HIPRTC_SUCCESS;
    if (!ok) {
        size_t n = 0;
        r.log_size(prog, &n);
        std::string log(n, '\0');
        if (n) r.log(prog, &log[0]);
        err = "hipRTC compile failed: " + log.substr(0, 2000);
    } else {
        size_t n = 0;
        ok = r.code_size(prog, &n) == HIPRTC_SUCCESS && n > 0;
        obj.assign(n, 0);
        ok = ok && r.code(prog, obj.data()) == HIPRTC_SUCCESS;
        if (!ok) err = "hipRTC returned no code";
    }
    r.destroy(&prog);
    if (ok) {
        dump(src, obj);
        cache_write(key, obj);
        std::lock_guard<std::mutex> lk(g_mu);
        g_objects.emplace(src, obj);
    }
    return ok;
}

std::shared_ptr<const Kernels> load(const Code &c, int t, int device, bool sp, std::string &err) {
    const std::string src = source(c, t, sp);
    if (src.empty()) {
        err = sp ? "sum-product needs a local position map and at most " + std::to_string(kSumProductMaxEdges) +
                       " edges per view"
                 : "no local position map";
        return nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_modules.find({device, src});
        if (it != g_modules.end()) return it->second;
    }
    std::vector<char> obj;
    if (!compile(src, obj, err)) return nullptr;
    auto k = std::make_shared<Kernels>();
    hipError_t e = hipModuleLoadData(&k->module, obj.data());
    for (int form = kCompressed; form <= kSumProduct && e == hipSuccess; ++form) {
        if ((form == kSumProduct) != sp) continue;
        if (form != kCompressed && c.t[t].eloc > kExplicitMaxEdges) continue;
        const std::string f = std::to_string(form);
        for (int pm = 0; pm < 2 && e == hipSuccess; ++pm)
            e = hipModuleGetFunction(&k->local[form - 1][pm], k->module, ("lead_spec_local_" + f + std::to_string(pm)).c_str());
        if (e == hipSuccess) e = hipModuleGetFunction(&k->global[form - 1], k->module, ("lead_spec_global_" + f).c_str());
        if (e == hipSuccess) e = hipModuleGetFunction(&k->round[form - 1], k->module, ("lead_spec_round_" + f).c_str());
        if (e == hipSuccess && form != kSumProduct && tile_fits(c, t))
            e = hipModuleGetFunction(&k->tile[form - 1], k->module, ("lead_spec_tile_" + f).c_str());
        if (e == hipSuccess && (form == kExplicit || form == kSumProduct))
            e = form == kExplicit && tile_fits(c, t)
                    ? hipModuleGetFunction(&k->tile_nf[form - 1], k->module, ("lead_spec_tile_" + f + "n").c_str())
                    : hipModuleGetFunction(&k->global_nf[form - 1], k->module, ("lead_spec_global_" + f + "n").c_str());
        if (e == hipSuccess) k->has[form - 1] = true;
        if (form == kExplicit) k->local_lds[form - 1][0] = sizeof(float) * 64 * (size_t)local_lds_edges(c.t[t]);
        for (int pm = 0; pm < 2 && e == hipSuccess; ++pm) {
            int nb = 0;
            if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->local[form - 1][pm], 64,
                                                                   k->local_lds[form - 1][pm]) == hipSuccess &&
                nb > 0)
                k->local_waves_per_cu[form - 1][pm] = nb;
        }
    }
    if (e == hipSuccess) e = hipModuleGetFunction(&k->local_osd, k->module, "lead_spec_local_osd");
    if (e == hipSuccess && osd_fits(c, t)) {
        e = hipModuleGetFunction(&k->osd, k->module, "lead_spec_osd");
        if (e == hipSuccess) e = hipModuleGetFunction(&k->osd_cs, k->module, "lead_spec_osd_cs");
        k->osd_wg = osd_workgroup(c, t);
    }
    if (e == hipSuccess && osd_big_fits(c, t)) {
        e = hipModuleGetFunction(&k->osd_big, k->module, "lead_spec_osd_big");
        if (e == hipSuccess) e = hipModuleGetFunction(&k->osd_big_cs, k->module, "lead_spec_osd_big_cs");
        k->osd_big_wg = osd_big_workgroup(c, t);
    }
    if (e != hipSuccess) {
        err = std::string("module load: ") + hipGetErrorString(e);
        if (k->module) (void)hipModuleUnload(k->module);
        return nullptr;
    }
    k->wg = workgroup_for(c.order);
    k->spw = k->wg / c.order;
    if (tile_fits(c, t)) {
        k->tile_shots = lead::kTileWG / c.order;
        k->tile_lds = tile_lds_bytes(c, t);
    }
    k->bperm = k->wg == 64;
    k->hybrid = hybrid_degree(c.t[t]) > 0;
    if (!k->bperm && lam_lds_fits(c, t)) {
        // across waves the per-shot kernels of form 1 (and of form 2 with
        // the mixed state) keep lambda' of the positions with sigma[j] >= j
        // in LDS (lead_spec::lam_in_lds)
        const int D2 = c.delta * c.delta;
        for (int j = 0; j < D2; ++j) k->lam_slots += c.t[t].sigma[j] >= j ? 1 : 0;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto ins = g_modules.emplace(std::make_pair(device, src), k);
    return ins.first->second;   // another thread may have loaded it first
}

int plain_state_words(const Code &c, int t) { return c.t[t].eloc + 4 * c.t[t].r; }

namespace {
std::map<std::pair<int, std::string>, std::shared_ptr<const FusedKernels>> g_fused;
}

void settle_fused_tiles(std::vector<FusedPart> &parts) {
    bool any = false, ok = true;
    for (FusedPart &p : parts) {
        p.tiles = p.tiles && p.form != kSumProduct && tile_fits(*p.code, p.t);
        any = any || p.tiles;
    }
    for (const FusedPart &p : parts) {
        if (p.tiles) continue;
        const TypeTables &tt = p.code->t[p.t];
        if (lead::kTileWG % workgroup_for(p.code->order) != 0 || (p.form == kSumProduct && tt.eloc > kTwoWaveMaxEdges))
            ok = false;
    }
    if (any && !ok)
        for (FusedPart &p : parts) p.tiles = false;
}

std::string fused_source(const std::vector<FusedPart> &parts, FusedKernels &kk, std::string &err) {
    if (parts.empty() || parts.size() > (size_t)lead::kFusedMax) {
        err = "a fused batch holds 1 to " + std::to_string(lead::kFusedMax) + " requests";
        return std::string();
    }
    FusedKernels *k = &kk;
    std::ostringstream o, structs, loc, glob;
    o << "#include \"lead_spec.hpp\"\n";
    std::map<std::string, std::string> names;   // struct text -> name
    std::vector<std::string> pname;
    bool whole_file = false;
    for (const FusedPart &p : parts) {
        const TypeTables &tt = p.code->t[p.t];
        const int D2 = p.code->delta * p.code->delta;
        if (tt.sigma.empty() || (int)tt.sigma.size() != D2 || p.form < kCompressed || p.form > kSumProduct ||
            (p.form != kCompressed && tt.eloc > kExplicitMaxEdges) || (p.form == kSumProduct && tt.eloc > kSumProductMaxEdges)) {
            err = "a request's code has no compiled kernels of its form";
            return std::string();
        }
        std::ostringstream body;
        emit_code_struct(body, *p.code, p.t, "@");
        std::string text = body.str();
        auto it = names.find(text);
        if (it == names.end()) {
            const std::string nm = "LeadCode" + std::to_string(names.size());
            it = names.emplace(text, nm).first;
            text.replace(text.find('@'), 1, nm);
            structs << text;
        }
        pname.push_back(it->second);
        if (p.form == kExplicit && p.pm == 0)
            k->local_lds = std::max(k->local_lds, sizeof(float) * 64 * (size_t)local_lds_edges(tt));
        if (p.tiles && (p.form == kSumProduct || !tile_fits(*p.code, p.t))) {
            err = "a request asks for the persistent kernel its code does not have";
            return std::string();
        }
        const int wg = p.tiles ? lead::kTileWG : workgroup_for(p.code->order);
        k->wg = std::max(k->wg, wg);
        whole_file = whole_file || (p.form == kSumProduct && tt.eloc > kTwoWaveMaxEdges);
    }
    // a module with persistent workgroups runs eight waves per workgroup,
    // one workgroup per compute unit (two waves per SIMD)
    bool any_tiles = false;
    for (const FusedPart &p : parts) any_tiles = any_tiles || p.tiles;
    if (any_tiles && whole_file) {
        err = "the persistent kernel and a whole-register-file kernel cannot share a workgroup shape";
        return std::string();
    }
    o << structs.str();
    o << "extern \"C\" __global__ void __launch_bounds__(64) lead_fused_local(lead::FusedArgs f) {\n";
    for (size_t i = 0; i < parts.size(); ++i)
        o << "    if (!f.it[" << i << "].a.global_only) lead_spec::local_body<" << pname[i] << ", " << parts[i].pm << ", "
          << parts[i].form << ">(f.it[" << i << "].a, f.it[" << i << "].w);\n";
    o << "}\n";
    o << "extern \"C\" __global__ void __launch_bounds__(" << k->wg << (whole_file || any_tiles ? "" : ", 2")
      << ") lead_fused_global(lead::FusedArgs f) {\n"
         "    extern __shared__ float lds_f[];\n"
         "    const int64_t b = blockIdx.x;\n";
    for (size_t i = 0; i < parts.size(); ++i) {
        const FusedPart &p = parts[i];
        const Code &c = *p.code;
        const TypeTables &tt = c.t[p.t];
        const int D2 = c.delta * c.delta, wg = workgroup_for(c.order);
        if (p.tiles) {
            // the whole workgroup, persistent, for this request
            k->sub.push_back(1);
            k->lds_words.push_back(0);
            k->spw.push_back(1);
            k->tile_shots.push_back(lead::kTileWG / c.order);
            k->lds_bytes = std::max(k->lds_bytes, tile_lds_bytes(c, p.t));
            o << "    " << (i ? "else " : "") << "if (b < f.first[" << i + 1 << "]) {\n"
              << "        lead_spec::global_tile_body<" << pname[i] << ", " << p.form << ">(f.it[" << i << "].a, f.it["
              << i << "].w, f.it[" << i << "].x);\n"
              << "    }\n";
            continue;
        }
        if (k->wg % wg != 0) {
            err = "the codes' per-shot workgroups (" + std::to_string(wg) + " and " + std::to_string(k->wg) +
                  " lanes) do not divide one another";
            return std::string();
        }
        const bool bperm = wg == 64;
        const int spw = wg / c.order, sub = k->wg / wg;
        int slots = 0;
        if (!bperm && lam_lds_fits(c, p.t))
            for (int j = 0; j < D2; ++j) slots += tt.sigma[j] >= j ? 1 : 0;
        const bool lam_in_lds = p.form == kCompressed || (p.form == kExplicit && hybrid_degree(tt) > 0);
        const int words = (bperm ? 0 : D2 * wg) + (lam_in_lds ? slots * wg : 0) + 9 * spw + spw * ((c.n + 31) / 32);
        k->sub.push_back(sub);
        k->lds_words.push_back(words);
        k->spw.push_back(spw);
        k->tile_shots.push_back(0);
        k->lds_bytes = std::max(k->lds_bytes, sizeof(float) * (size_t)words * sub);
        o << "    " << (i ? "else " : "") << "if (b < f.first[" << i + 1 << "]) {\n";
        if (sub == 1)   // the block is the workgroup: the launch's lane and LDS, as in the per-code kernel
            o << "        const lead_spec::Blk blk{b - f.first[" << i << "], (int)threadIdx.x, lds_f};\n";
        else
            o << "        const int sb = (int)threadIdx.x / " << wg << ";\n"
              << "        const lead_spec::Blk blk{(b - f.first[" << i << "]) * " << sub << " + sb, (int)threadIdx.x - sb * "
              << wg << ", lds_f + sb * " << words << "};\n";
        o
          << "        lead_spec::global_body<" << pname[i] << ", " << wg << ", " << (bperm ? "true" : "false") << ", "
          << p.form << ">(f.it[" << i << "].a, f.it[" << i << "].w, f.it[" << i << "].x, lead::PlainArgs{}, blk);\n"
          << "    }\n";
    }
    o << "}\n";
    return o.str();
}

std::shared_ptr<const FusedKernels> load_fused(const std::vector<FusedPart> &parts, int device, std::string &err) {
    auto k = std::make_shared<FusedKernels>();
    const std::string src = fused_source(parts, *k, err);
    if (src.empty()) return nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_fused.find({device, src});
        if (it != g_fused.end()) return it->second;
    }
    std::vector<char> obj;
    if (!compile(src, obj, err)) return nullptr;
    hipError_t e = hipModuleLoadData(&k->module, obj.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&k->local, k->module, "lead_fused_local");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->global, k->module, "lead_fused_global");
    if (e != hipSuccess) {
        err = std::string("fused module load: ") + hipGetErrorString(e);
        if (k->module) (void)hipModuleUnload(k->module);
        return nullptr;
    }
    int nb = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->local, 64, 0) == hipSuccess && nb > 0)
        k->local_waves_per_cu = nb;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_fused.emplace(std::make_pair(device, src), k).first->second;
}

void partner_tables(const Code &c, int t, std::vector<uint32_t> &pv, std::vector<uint64_t> &fown) {
    const TypeTables &tt = c.t[t];
    const int D2 = c.delta * c.delta, NP = (D2 + 1) / 2, N = c.order;
    pv.assign((size_t)N * NP, 0u);
    fown.assign((size_t)N, 0ull);
    for (int v = 0; v < N; ++v)
        for (int j = 0; j < D2; ++j) {
            const int s = v * D2 + j;
            const uint32_t vp = (uint32_t)(tt.partner[s] / D2);
            pv[(size_t)v * NP + j / 2] |= vp << (16 * (j & 1));
            if (!tt.sigma.empty() && tt.sigma[j] == j && tt.owned[s]) fown[v] |= 1ull << j;
        }
}

}  // namespace jit
}  // namespace lead
