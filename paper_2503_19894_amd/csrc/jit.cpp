// Dynamic kernels (Sec. IV-A): one kernel per fused gate, generated at run
// time from the gate's matrix and compiled for gfx950 with hipRTC.
//
// The generated kernel is the direct gather (lanes take consecutive group
// indices, work item = (group, non-identity block)) with everything the
// gate's analysis knows baked in as constants: target masks, block offsets
// and the matrix entries themselves as immediates (cast to the state dtype).
// Per entry, exact zeros are dropped, entries +-1 and +-i become additions,
// and within an output row the amplitudes that share a coefficient up to
// sign are summed before the one multiplication (element sharing).  Gates
// whose blocks are larger than 16 x 16 run with the library's kernels.
#include <hip/hiprtc.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>

#include "internal.hpp"

namespace cast {

constexpr int kJitMaxD = 4;

struct JitModule {
    std::vector<char> code;          // code object from hipRTC
    std::vector<std::string> names;  // kernel per plan ("" = library kernel)
    hipModule_t mod = nullptr;       // loaded on first apply
    std::vector<hipFunction_t> fn;
    double compile_ms = 0;
    int kernels = 0;
};

void jit_free(JitModule *j) {
    if (!j) return;
    if (j->mod) (void)hipModuleUnload(j->mod);
    delete j;
}

namespace {

std::string hex64(uint64_t v) {
    char b[32];
    std::snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}

// Exact literal of a value in the state dtype.
std::string lit(double v, bool f32) {
    char b[64];
    if (f32) std::snprintf(b, sizeof b, "%af", (double)(float)v);
    else std::snprintf(b, sizeof b, "%a", v);
    return b;
}

// r + i m for one output row: sum over coefficient classes (equal up to
// sign) of coef * (sum of +-amplitudes).
void emit_row(std::string &s, const std::vector<cplx> &row, bool f32, const std::string &T, int r) {
    struct Cls {
        double a, b;                        // canonical coefficient (first nonzero part > 0)
        std::vector<std::pair<int, int>> t; // (column, sign)
    };
    std::vector<Cls> cls;
    for (size_t c = 0; c < row.size(); ++c) {
        double a = row[c].real(), b = row[c].imag();
        if (f32) a = (float)a, b = (float)b;
        if (a == 0 && b == 0) continue;
        int sg = (a > 0 || (a == 0 && b > 0)) ? 1 : -1;
        const double ca = sg * a, cb = sg * b;
        bool found = false;
        for (Cls &k : cls)
            if (k.a == ca && k.b == cb) {
                k.t.push_back({(int)c, sg});
                found = true;
                break;
            }
        if (!found) cls.push_back({ca, cb, {{(int)c, sg}}});
    }
    s += "        {\n          " + T + " ar = 0, ai = 0;\n";
    for (const Cls &k : cls) {
        std::string sx, sy;
        for (auto [c, sg] : k.t) {
            sx += (sg > 0 ? (sx.empty() ? "" : " + ") : " - ") + std::string("v") + std::to_string(c) + ".x";
            sy += (sg > 0 ? (sy.empty() ? "" : " + ") : " - ") + std::string("v") + std::to_string(c) + ".y";
        }
        s += "          { const " + T + " sx = " + sx + ", sy = " + sy + ";\n";
        const std::string A = lit(k.a, f32), B = lit(k.b, f32), NB = lit(-k.b, f32);
        if (k.b == 0 && k.a == 1) s += "            ar += sx; ai += sy; }\n";
        else if (k.a == 0 && k.b == 1) s += "            ar -= sy; ai += sx; }\n";
        else if (k.b == 0) s += "            ar = FMA(" + A + ", sx, ar); ai = FMA(" + A + ", sy, ai); }\n";
        else if (k.a == 0) s += "            ar = FMA(" + NB + ", sy, ar); ai = FMA(" + B + ", sx, ai); }\n";
        else
            s += "            ar = FMA(" + A + ", sx, ar); ar = FMA(" + NB + ", sy, ar); ai = FMA(" + A +
                 ", sy, ai); ai = FMA(" + B + ", sx, ai); }\n";
    }
    s += "          V o; o.x = ar; o.y = ai; psi[b ^ O" + std::to_string(r) + "] = o;\n        }\n";
}

std::string kernel_source(const PassPlan &p, int n, bool f32, const std::string &name) {
    const std::string T = f32 ? "float" : "double";
    const int k = p.k, d = p.d, N = 1 << d;
    const int lng = n - k;
    const size_t nblk = p.blk.size();
    // physical offset of each virtual basis vector
    uint64_t off[kMaxK];
    for (int i = 0; i < k; ++i) {
        uint64_t o = 0;
        for (int s2 = 0; s2 < k; ++s2)
            if ((p.L[i] >> s2) & 1u) o |= 1ull << p.q[s2];
        off[i] = o;
    }
    std::string s = "extern \"C\" __global__ void __launch_bounds__(256) " + name + "(V *__restrict__ psi) {\n";
    s += "  const unsigned long long items = " + hex64((uint64_t)nblk << lng) + ";\n";
    s += "  for (unsigned long long it = blockIdx.x * 256ull + threadIdx.x; it < items;"
         " it += (unsigned long long)gridDim.x * 256ull) {\n";
    s += "    const unsigned bs = (unsigned)(it >> " + std::to_string(lng) + ");\n";
    s += "    unsigned long long g = it & " + hex64((1ull << lng) - 1) + ";\n";
    for (int i = 0; i < k; ++i) {
        const std::string m = hex64((1ull << p.q[i]) - 1);
        s += "    g = ((g & ~" + m + ") << 1) | (g & " + m + ");\n";
    }
    for (int c = 0; c < N; ++c) {
        uint64_t o = 0;
        for (int i = 0; i < d; ++i)
            if ((c >> i) & 1) o ^= off[i];
        s += "    const unsigned long long O" + std::to_string(c) + " = " + hex64(o) + ";\n";
    }
    s += "    switch (bs) {\n";
    for (size_t bi = 0; bi < nblk; ++bi) {
        uint64_t bo = 0;
        for (int j = 0; j < k - d; ++j)
            if ((p.blk[bi] >> j) & 1u) bo ^= off[d + j];
        s += "    case " + std::to_string(bi) + ": {\n";
        s += "      const unsigned long long b = g ^ " + hex64(bo) + ";\n";
        for (int c = 0; c < N; ++c)
            s += "      const V v" + std::to_string(c) + " = psi[b ^ O" + std::to_string(c) + "];\n";
        for (int r = 0; r < N; ++r) {
            std::vector<cplx> row(p.mat.begin() + (bi * N + r) * N, p.mat.begin() + (bi * N + r + 1) * N);
            emit_row(s, row, f32, T, r);
        }
        s += "    } break;\n";
    }
    s += "    }\n  }\n}\n";
    return s;
}

cast_status compile(const cast_fused &f, cast_dtype dt, JitModule **out) {
    const bool f32 = dt == CAST_C64;
    auto t0 = std::chrono::steady_clock::now();
    auto *j = new JitModule;
    j->names.assign(f.plans.size(), "");
    std::string src = f32 ? "typedef float V __attribute__((ext_vector_type(2)));\n#define FMA __builtin_fmaf\n"
                          : "typedef double V __attribute__((ext_vector_type(2)));\n#define FMA __builtin_fma\n";
    for (size_t i = 0; i < f.plans.size(); ++i) {
        const PassPlan &p = f.plans[i];
        if (p.identity() || p.d > kJitMaxD) continue;
        j->names[i] = "cast_jit_" + std::to_string(i);
        src += kernel_source(p, f.n, f32, j->names[i]);
        ++j->kernels;
    }
    if (j->kernels) {
        hiprtcProgram prog;
        if (hiprtcCreateProgram(&prog, src.c_str(), "cast_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
            jit_free(j);
            return fail(CAST_EHIP, "hiprtcCreateProgram failed");
        }
        const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
                              "-packed-fp32-ops"};
        const hiprtcResult rc = hiprtcCompileProgram(prog, 6, opts);
        if (rc != HIPRTC_SUCCESS) {
            size_t ls = 0;
            hiprtcGetProgramLogSize(prog, &ls);
            std::string log(ls, '\0');
            if (ls) hiprtcGetProgramLog(prog, &log[0]);
            hiprtcDestroyProgram(&prog);
            jit_free(j);
            return fail(CAST_EHIP, std::string("hipRTC compile failed: ") + hiprtcGetErrorString(rc) + "\n" +
                                       log.substr(0, 2000));
        }
        size_t sz = 0;
        hiprtcGetCodeSize(prog, &sz);
        j->code.resize(sz);
        hiprtcGetCode(prog, j->code.data());
        hiprtcDestroyProgram(&prog);
    }
    j->compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = j;
    return CAST_OK;
}

cast_status prepare(const cast_fused *fc, cast_dtype dt, bool device, JitModule **out) {
    if (!fc) return fail(CAST_EINVAL, "fused list is NULL");
    if (dt != CAST_C64 && dt != CAST_C128) return fail(CAST_EINVAL, "bad dtype");
    cast_fused *f = const_cast<cast_fused *>(fc);
    JitModule *&j = f->jit[dt];
    if (!j) {
        if (cast_status rc = compile(*f, dt, &j)) return rc;
    }
    if (device) {
        if (!f->dev[dt].ptr && !f->plans.empty()) {
            if (cast_status rc = upload_plans(f->plans, dt, &f->dev[dt], &f->dev_off[dt])) return rc;
        }
        if (!j->mod && j->kernels) {
            CAST_HIP_TRY(hipModuleLoadData(&j->mod, j->code.data()));
            j->fn.assign(f->plans.size(), nullptr);
            for (size_t i = 0; i < f->plans.size(); ++i)
                if (!j->names[i].empty()) CAST_HIP_TRY(hipModuleGetFunction(&j->fn[i], j->mod, j->names[i].c_str()));
        }
    }
    *out = j;
    return CAST_OK;
}

cast_status launch(cast_sv *sv, const cast_fused *f, const JitModule &j, size_t i) {
    const PassPlan &p = f->plans[i];
    if (p.identity()) return CAST_OK;
    if (j.fn.empty() || !j.fn[i]) {
        const size_t rsz = sv->dt == CAST_C128 ? 8 : 4;
        const void *dm = (const char *)f->dev[sv->dt].ptr + f->dev_off[sv->dt][i] * rsz;
        return launch_pass(sv->data, sv->n, sv->dt, p, dm, sv->stream);
    }
    const uint64_t items = (uint64_t)p.blk.size() << (sv->n - p.k);
    uint64_t grid = (items + 255) / 256;
    if (grid > (uint64_t)tuning().max_grid[sv->dt]) grid = tuning().max_grid[sv->dt];
    void *psi = sv->data;
    void *args[] = {&psi};
    CAST_HIP_TRY(hipModuleLaunchKernel(j.fn[i], (unsigned)grid, 1, 1, 256, 1, 1, 0, sv->stream, args, nullptr));
    return CAST_OK;
}

}  // namespace
}  // namespace cast

using namespace cast;

extern "C" {

cast_status jit_compile(const cast_fused *f, cast_dtype dt, int *n_kernels, double *compile_ms) {
    JitModule *j;
    if (cast_status rc = prepare(f, dt, false, &j)) return rc;
    if (n_kernels) *n_kernels = j->kernels;
    if (compile_ms) *compile_ms = j->compile_ms;
    return CAST_OK;
}

cast_status apply_circuit_jit(cast_sv *sv, const cast_fused *f) {
    if (!sv || !sv->data) return fail(CAST_EINVAL, "state is NULL");
    if (!f) return fail(CAST_EINVAL, "fused list is NULL");
    if (f->n != sv->n) return fail(CAST_EINVAL, "fused list was built for a different qubit count");
    JitModule *j;
    if (cast_status rc = prepare(f, sv->dt, true, &j)) return rc;
    for (size_t i = 0; i < f->plans.size(); ++i)
        if (cast_status rc = launch(sv, f, *j, i)) return rc;
    return CAST_OK;
}

cast_status apply_circuit_jit_timed(cast_sv *sv, const cast_fused *f, float *pass_ms) {
    if (!sv || !sv->data) return fail(CAST_EINVAL, "state is NULL");
    if (!f || !pass_ms) return fail(CAST_EINVAL, "NULL argument");
    if (f->n != sv->n) return fail(CAST_EINVAL, "fused list was built for a different qubit count");
    JitModule *j;
    if (cast_status rc = prepare(f, sv->dt, true, &j)) return rc;
    const size_t np = f->plans.size();
    std::vector<hipEvent_t> ev(np + 1, nullptr);
    cast_status rc = CAST_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(CAST_EHIP, "hipEventCreate failed");
    if (!rc && hipEventRecord(ev[0], sv->stream) != hipSuccess) rc = fail(CAST_EHIP, "hipEventRecord failed");
    for (size_t i = 0; i < np && !rc; ++i) {
        rc = launch(sv, f, *j, i);
        if (!rc && hipEventRecord(ev[i + 1], sv->stream) != hipSuccess) rc = fail(CAST_EHIP, "hipEventRecord failed");
    }
    if (!rc && hipEventSynchronize(ev[np]) != hipSuccess) rc = fail(CAST_EHIP, "hipEventSynchronize failed");
    for (size_t i = 0; i < np && !rc; ++i)
        if (hipEventElapsedTime(&pass_ms[i], ev[i], ev[i + 1]) != hipSuccess)
            rc = fail(CAST_EHIP, "hipEventElapsedTime failed");
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

}  // extern "C"
