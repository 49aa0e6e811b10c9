// Walk programs through the C ABI: a program's source is compiled at run time
// (hipRTC) against program_rt.hpp, loaded as a module and launched with the
// same arguments as a built-in walk.
#include <dlfcn.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "program_rt.hpp"
#include "trw_internal.hpp"

struct trw_program_s {
    hipModule_t module = nullptr;
    hipFunction_t kernel = nullptr;
    uint32_t kind = 0;
    int device = 0;
};

namespace trw {
namespace {

trw_status pfail(trw_status st, const std::string &m) {
    set_error(m);
    return st;
}

// The directory holding program_rt.hpp: csrc/ next to this library.
std::string runtime_include_dir() {
    Dl_info info{};
    if (dladdr(reinterpret_cast<void *>(&runtime_include_dir), &info) && info.dli_fname) {
        std::string lib(info.dli_fname);
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/csrc";
    }
    return "csrc";
}

// The program's source, then the kernel and its kind for the loader.
std::string full_source(const char *source) {
    std::string s = "#include \"program_rt.hpp\"\n";
    s += source;
    s += "\nextern \"C\" __global__ void __launch_bounds__(256) trw_program_kernel(trw_prog::Args a) {\n"
         "    trw_prog::run<TrwProgram>(a);\n}\n"
         "extern \"C\" __device__ __constant__ unsigned int trw_program_kind = TrwProgram::kind;\n";
    return s;
}

trw_status compile(const char *source, const std::string &arch, std::vector<char> *code) {
    const std::string src = full_source(source);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "trw_program.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return pfail(TRW_E_DEVICE, "hiprtcCreateProgram failed");
    const std::string arch_opt = "--offload-arch=" + arch;
    const std::string inc_opt = "-I" + runtime_include_dir();
    const char *opts[] = {arch_opt.c_str(), inc_opt.c_str(), "-O3", "-std=c++17",
                          // no packed FP32 instructions (as the library itself)
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        (void)hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) (void)hiprtcGetProgramLog(prog, &log[0]);
        (void)hiprtcDestroyProgram(&prog);
        return pfail(TRW_E_INVALID, "walk program does not compile:\n" + log);
    }
    size_t n = 0;
    if (code) {
        (void)hiprtcGetCodeSize(prog, &n);
        code->resize(n);
        (void)hiprtcGetCode(prog, code->data());
    }
    (void)hiprtcDestroyProgram(&prog);
    return TRW_OK;
}

__global__ void k_zero_head(unsigned long long *p) { *p = 0; }

}  // namespace
}  // namespace trw

using namespace trw;

extern "C" {

trw_status trw_program_check(const char *source, const char *arch) {
    if (!source || !arch) return pfail(TRW_E_INVALID, "source / arch is NULL");
    return compile(source, arch, nullptr);
}

trw_status trw_program_create(const char *source, trw_program *out) {
    if (!source || !out) return pfail(TRW_E_INVALID, "source / out is NULL");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return pfail(TRW_E_DEVICE, "no HIP device");
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    std::vector<char> code;
    trw_status st = compile(source, arch, &code);
    if (st != TRW_OK) return st;
    auto *p = new (std::nothrow) trw_program_s();
    if (!p) return pfail(TRW_E_INVALID, "out of host memory");
    p->device = dev;
    hipError_t e = hipModuleLoadData(&p->module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&p->kernel, p->module, "trw_program_kernel");
    hipDeviceptr_t kind_ptr = nullptr;
    size_t kind_bytes = 0;
    if (e == hipSuccess) e = hipModuleGetGlobal(&kind_ptr, &kind_bytes, p->module, "trw_program_kind");
    if (e == hipSuccess) e = hipMemcpyDtoH(&p->kind, kind_ptr, sizeof(uint32_t));
    if (e != hipSuccess) {
        if (p->module) (void)hipModuleUnload(p->module);
        delete p;
        return pfail(TRW_E_DEVICE, std::string("walk program load: ") + hipGetErrorString(e));
    }
    if (p->kind > trw_prog::STATIC_REJ) {
        (void)hipModuleUnload(p->module);
        delete p;
        return pfail(TRW_E_INVALID, "TrwProgram::kind is not a sampling method");
    }
    *out = p;
    return TRW_OK;
}

trw_status trw_program_kind(trw_program p, uint32_t *kind) {
    if (!p || !kind) return pfail(TRW_E_INVALID, "program / kind is NULL");
    *kind = p->kind;
    return TRW_OK;
}

trw_status trw_program_walk(trw_program prog, trw_graph g, trw_table table, const trw_program_params *pp,
                            const int32_t *d_sources, uint64_t nq, uint64_t qid_base, int32_t *d_paths,
                            uint64_t path_stride, uint32_t *d_lengths, uint8_t *d_status, void *d_ws,
                            size_t ws_bytes, trw_stream_t stream) {
    if (!prog || !g || !pp) return pfail(TRW_E_INVALID, "program / graph / params is NULL");
    if (pp->max_len == 0 || pp->max_len > 65535) return pfail(TRW_E_INVALID, "max_len must be in 1..65535");
    if (nq >= (uint64_t(1) << 32)) return pfail(TRW_E_INVALID, "nq must be < 2^32");
    if (path_stride < (uint64_t)pp->max_len + 1) return pfail(TRW_E_INVALID, "path_stride < max_len + 1");
    const GraphDev &gd = graph_dev(g);
    trw_prog::Args a{};
    a.g.row_ptr = gd.row_ptr;
    a.g.col = gd.col;
    a.g.weight = gd.weight;
    a.g.label = gd.label;
    a.g.n = gd.n;
    a.g.m = gd.m;
    a.g.symmetric = gd.symmetric ? 1u : 0u;
    const void *buf = nullptr;
    trw_graph tg = nullptr;
    if (prog->kind == trw_prog::STATIC_ALIAS || prog->kind == trw_prog::STATIC_ITS ||
        prog->kind == trw_prog::STATIC_REJ) {
        const uint32_t want = prog->kind == trw_prog::STATIC_ALIAS ? TRW_S_ALIAS
                              : prog->kind == trw_prog::STATIC_ITS ? TRW_S_ITS : TRW_S_REJ;
        if (!table_view(table, want, &buf, &tg) || tg != g)
            return pfail(TRW_E_INVALID, "a STATIC_ALIAS / STATIC_ITS / STATIC_REJ program needs that table of this graph");
        if (want == TRW_S_ALIAS) {
            a.alias = static_cast<const uint4 *>(buf);
        } else if (want == TRW_S_ITS) {
            a.prefix = static_cast<const uint64_t *>(buf);
        } else {
            a.rej = static_cast<const uint4 *>(buf);
            a.g.pmax = reinterpret_cast<const uint32_t *>(static_cast<const char *>(buf) + rej_records_bytes(gd.m));
        }
    } else if (table) {
        // a NAIVE or dynamic program: an edge index (for is_neighbor) or a REJ
        // table (for the per-vertex bound p*, Walker::pm)
        if (table_view(table, kEdgeIndexKind, &buf, &tg) && tg == g) {
            a.g.eset = reinterpret_cast<const unsigned long long *>(static_cast<const char *>(buf) +
                                                                    edge_index_records_bytes(gd.m));
            a.g.eset_mask = eset_slots(gd.m) - 1;
        } else if (table_view(table, TRW_S_REJ, &buf, &tg) && tg == g) {
            a.g.pmax = reinterpret_cast<const uint32_t *>(static_cast<const char *>(buf) + rej_records_bytes(gd.m));
        } else {
            return pfail(TRW_E_INVALID,
                         "a NAIVE / dynamic program takes an edge index or a REJ table of this graph, or no table");
        }
    }
    if (nq == 0) return TRW_OK;
    if (!d_sources || !d_paths || !d_lengths || !d_status)
        return pfail(TRW_E_INVALID, "sources / paths / lengths / status is NULL");
    if (!d_ws || ws_bytes < 8 || (reinterpret_cast<uintptr_t>(d_ws) & 7))
        return pfail(TRW_E_INVALID, "workspace must hold 8 bytes, 8-byte aligned");
    a.sources = d_sources;
    a.nq = (uint32_t)nq;
    a.chunk = 128;
    a.qid_base = qid_base;
    a.paths = d_paths;
    a.stride = path_stride;
    a.lengths = d_lengths;
    a.status = d_status;
    a.head = static_cast<unsigned long long *>(d_ws);
    a.p.max_len = pp->max_len;
    a.p.seed = pp->seed;
    std::memcpy(a.p.user, pp->user, sizeof(a.p.user));
    auto s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_head, dim3(1), dim3(1), 0, s, a.head);
    const DeviceInfo di = device_info();
    const uint64_t waves = (nq + 63) / 64;
    // Launch shape measured on MI355X: static programs (one random read per
    // move) peak at 2 workgroups per CU, dynamic ones at full occupancy.
    const bool static_kind = prog->kind <= trw_prog::STATIC_ITS || prog->kind == trw_prog::STATIC_REJ;
    const uint64_t per_cu = static_kind ? 2 : 8;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((waves + 3) / 4, (uint64_t)di.num_cus * per_cu));
    void *args[] = {&a};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipModuleLaunchKernel(prog->kernel, blocks, 1, 1, 256, 1, 1, 0, s, args, nullptr);
    if (e != hipSuccess) return pfail(TRW_E_DEVICE, std::string("walk program launch: ") + hipGetErrorString(e));
    return TRW_OK;
}

trw_status trw_program_destroy(trw_program p) {
    if (!p) return TRW_OK;
    if (p->module) (void)hipModuleUnload(p->module);
    delete p;
    return TRW_OK;
}

}  // extern "C"
