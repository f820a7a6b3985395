// Plan-specialized matvec kernels, generated as HIP source and compiled with hiprtc for the current
// device.  The generated kernel applies the same map as the generic one (target-driven gather, Sec. II;
// digits by Eq. decode; channels by Eqs. src_digit_two_site / sourceoffset; ladder factors of App. A,
// App. B, App. C) but with the plan's structure baked in:
//
//  * the index space is tiled: the low sites [k_in, N) form an inner block of T_in consecutive rows,
//    one thread per inner row; the outer sites' digits are the same for the whole tile, so they are
//    computed once per tile on the scalar unit from the tile number (compile-time divisors);
//  * a channel touching only outer sites is admissible for the whole tile or for none of it: one
//    uniform branch, one uniform coefficient;
//  * a channel touching inner sites gets its per-row factor (0 where inadmissible) once per thread,
//    kept in a register across all the tiles the persistent block visits;
//  * x is read through a buffer descriptor: the per-row part of every address (r * element size) is one
//    register fixed for the whole kernel and the per-channel part (F0 - Delta) is a scalar, so the
//    gather issues no vector address arithmetic; y is written with non-temporal stores so it does not
//    evict x from the caches;
//  * tiles are dealt to blocks so that the 8 XCDs each sweep a contiguous stretch of tiles at a time.
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <sstream>

#include "mrmf_internal.h"

namespace mrmf {
namespace {

std::string lit(double v, bool f32) {
    char buf[64];
    if (f32)
        std::snprintf(buf, sizeof buf, "%af", static_cast<double>(static_cast<float>(v)));
    else
        std::snprintf(buf, sizeof buf, "%a", v);
    return buf;
}

// Factor <n|O|n - q> of a local operator at target digit n, 0 where the source digit is outside 0..d-1.
std::vector<double> factor_table(const mrmf_plan_t* p, int site, int op) {
    const int d = p->d[site], tab = p->tab[site];
    std::vector<double> t(d, 0.0);
    for (int n = 0; n < d; ++n) {
        switch (op) {
            case MRMF_OP_Z: t[n] = p->val[tab + n]; break;
            case MRMF_OP_Z2: t[n] = p->val[tab + n] * p->val[tab + n]; break;
            case MRMF_OP_RAISE: t[n] = n >= 1 ? p->up[tab + n] : 0.0; break;
            default: t[n] = n <= d - 2 ? p->up[tab + n + 1] : 0.0; break;
        }
    }
    return t;
}

// integer admissibility test of a uniform digit for a ladder operator ("" when always admissible)
std::string adm_expr(const mrmf_plan_t* p, int site, int op) {
    if (op == MRMF_OP_RAISE) return "n" + std::to_string(site) + " >= 1u";
    if (op == MRMF_OP_LOWER) return "n" + std::to_string(site) + " <= " + std::to_string(p->d[site] - 2) + "u";
    return "";
}

struct Gen {
    const mrmf_plan_t* p;
    bool f32;
    int k_in, T_in, block;
    int64_t n_tiles;
    std::set<std::pair<int, int>> arrays;  // (site, op) tables emitted as constant arrays
    std::set<std::string> arrays_named;
    std::ostringstream pre;                // constant arrays

    bool inner(int site) const { return site >= k_in; }
    // 0: every site of the term inner, 1: every site outer, 2: one inner and one outer site
    int cls(int a, int b) const {
        if (b < 0) return inner(a) ? 0 : 1;
        if (inner(a) && inner(b)) return 0;
        if (!inner(a) && !inner(b)) return 1;
        return 2;
    }

    // constant array holding a table (emitted once)
    // all constant tables live in one array K[] (one base address for every scalar load);
    // carray returns the offset of a table, appending it on first use
    std::map<std::string, size_t> pool_index;
    std::vector<double> pool;
    size_t carray(const std::string& name, const std::vector<double>& t) {
        auto it = pool_index.find(name);
        if (it != pool_index.end()) return it->second;
        const size_t off = pool.size();
        pool.insert(pool.end(), t.begin(), t.end());
        pool_index[name] = off;
        return off;
    }
    // factor of (site, op) at a tile-uniform digit: a scalar load from the constant pool
    std::string fac_uni(int site, int op) {
        const size_t off = carray("U" + std::to_string(site) + "_" + std::to_string(op), factor_table(p, site, op));
        return "K[" + std::to_string(off) + "u + n" + std::to_string(site) + "]";
    }
    // product of the two factors of an outer two-site term, one table indexed by both digits
    std::string fac_uni2(int a, int opa, int b, int opb) {
        const std::vector<double> ta = factor_table(p, a, opa), tb = factor_table(p, b, opb);
        std::vector<double> t(ta.size() * tb.size());
        for (size_t i = 0; i < ta.size(); ++i)
            for (size_t j = 0; j < tb.size(); ++j) t[i * tb.size() + j] = ta[i] * tb[j];
        const std::string name = "P" + std::to_string(a) + "_" + std::to_string(opa) + "_" + std::to_string(b) + "_" +
                                 std::to_string(opb);
        const size_t off = carray(name, t);
        return "K[" + std::to_string(off) + "u + n" + std::to_string(a) + " * " + std::to_string(tb.size()) + "u + n" +
               std::to_string(b) + "]";
    }
    // expression for the factor of (site, op) at the digit variable n<site>
    std::string fac(int site, int op) {
        const std::vector<double> t = factor_table(p, site, op);
        const std::string n = "n" + std::to_string(site);
        const int d = static_cast<int>(t.size());
        if (d <= 4) {
            std::string e = lit(t[d - 1], f32);
            for (int i = d - 2; i >= 0; --i) e = "(" + n + " == " + std::to_string(i) + "u ? " + lit(t[i], f32) + " : " + e + ")";
            return e;
        }
        const std::string name = "T" + std::to_string(site) + "_" + std::to_string(op);
        if (!arrays.count({site, op})) {
            arrays.insert({site, op});
            pre << "__constant__ R " << name << "[" << d << "] = {";
            for (int i = 0; i < d; ++i) pre << (i ? ", " : "") << lit(t[i], f32);
            pre << "};\n";
        }
        return name + "[" + n + "]";
    }

    std::string source() {
        const mrmf_plan_t& P = *p;
        const int SZ = f32 ? 8 : 16;
        const int64_t shift = int64_t(T_in) * SZ;
        const int nch = static_cast<int>(P.chans.size());
        const int ndg = static_cast<int>(P.diags.size());
        std::ostringstream o;
        std::set<int> used_sites, used_params;
        for (const auto& c : P.chans) {
            used_sites.insert(c.a);
            if (c.b >= 0) used_sites.insert(c.b);
            used_params.insert(c.param);
        }
        for (const auto& g : P.diags) {
            used_sites.insert(g.a);
            if (g.b >= 0) used_sites.insert(g.b);
            used_params.insert(g.param);
        }
        bool complex_w = false;
        for (const auto& c : P.chans) complex_w |= c.wi != 0.0;
        for (const auto& g : P.diags) complex_w |= g.wi != 0.0;
        // LDS halo: inner channels read the tile's own x at r - Delta, Delta < T_in
        int64_t pad = 0;
        for (const auto& c : P.chans)
            if (cls(c.a, c.b) == 0) pad = std::max<int64_t>(pad, c.delta < 0 ? -c.delta : c.delta);
        const bool use_lds = pad > 0;
        const int64_t rows_lds = T_in + 2 * pad + 1;  // halo, tile, halo, one slot idle lanes write to
        std::vector<int> cI, cO, cM;  // channels by class: inner, outer, mixed
        for (int c = 0; c < nch; ++c) {
            const int k = cls(P.chans[c].a, P.chans[c].b);
            (k == 0 ? cI : k == 1 ? cO : cM).push_back(c);
        }

        o << "extern \"C\" __global__ __launch_bounds__(" << block << ") void mrmf_spec(const R* __restrict__ theta,\n"
          << "    const C* __restrict__ x, C* __restrict__ y, const int* __restrict__ skip) {\n"
          << "  if (skip != nullptr && *skip != 0) return;\n";
        if (use_lds)
            o << "  __shared__ C lds[2 * " << rows_lds << "];\n"
              << "  for (unsigned i = threadIdx.x; i < " << pad << "u; i += " << block << "u) {\n"
              << "    const C z = {(R)0, (R)0};\n"
              << "    lds[i] = z; lds[" << pad + T_in << "u + i] = z; lds[" << rows_lds << "u + i] = z; lds["
              << rows_lds + pad + T_in << "u + i] = z;\n  }\n";
        // lanes past the tile (r >= T_in) run the same code: their loads and stores use an out-of-range
        // buffer offset (no memory access, loads return 0) and their coefficients are 0
        o << "  const unsigned r0 = threadIdx.x;\n"
          << "  const bool act = r0 < " << T_in << "u;\n"
          << "  const unsigned r = act ? r0 : 0u;\n"
          << "  const unsigned OOB = 0x80000000u;\n"
          << "  const unsigned voff = act ? r * " << SZ << "u : OOB;\n";
        for (int i : used_sites)
            if (inner(i))
                o << "  const unsigned n" << i << " = (r / " << P.M[i] << "u) % " << P.d[i] << "u;\n";
        for (int q : used_params) o << "  const R th" << q << " = theta[" << q << "];\n";
        for (int c = 0; c < nch; ++c) {
            const auto& ch = P.chans[c];
            o << "  const R cw" << c << "r = th" << ch.param << " * " << lit(ch.wr, f32) << ";\n";
            if (complex_w) o << "  const R cw" << c << "i = th" << ch.param << " * " << lit(ch.wi, f32) << ";\n";
        }
        for (int g = 0; g < ndg; ++g) {
            const auto& dg = P.diags[g];
            o << "  const R dw" << g << "r = th" << dg.param << " * " << lit(dg.wr, f32) << ";\n";
            if (complex_w) o << "  const R dw" << g << "i = th" << dg.param << " * " << lit(dg.wi, f32) << ";\n";
        }
        // per-thread parts, fixed for every tile: the inner diagonal, the inner factor of mixed terms,
        // and the whole coefficient of inner channels (0 where the source digit is out of range)
        o << "  R dIr = 0, dIi = 0;\n";
        for (int g = 0; g < ndg; ++g) {
            const auto& dg = P.diags[g];
            const int k = cls(dg.a, dg.b);
            if (k == 0) {
                std::string f = fac(dg.a, dg.opa);
                if (dg.b >= 0) f += " * " + fac(dg.b, dg.opb);
                o << "  { const R f = " << f << "; dIr += dw" << g << "r * f;";
                if (complex_w) o << " dIi += dw" << g << "i * f;";
                o << " }\n";
            } else if (k == 2) {
                const bool ia = inner(dg.a);
                o << "  const R fz" << g << " = " << fac(ia ? dg.a : dg.b, ia ? dg.opa : dg.opb) << ";\n";
            }
        }
        for (int c : cI) {
            const auto& ch = P.chans[c];
            std::string f = fac(ch.a, ch.opa);
            if (ch.b >= 0) f += " * " + fac(ch.b, ch.opb);
            o << "  const R k" << c << "r = act ? cw" << c << "r * " << f << " : (R)0;\n";
            if (complex_w) o << "  const R k" << c << "i = act ? cw" << c << "i * " << f << " : (R)0;\n";
        }
        for (int c : cM) {
            const auto& ch = P.chans[c];
            const bool ia = inner(ch.a);
            o << "  const R f" << c << " = " << fac(ia ? ch.a : ch.b, ia ? ch.opa : ch.opb) << ";\n"
              << "  const unsigned vo" << c << " = (f" << c << " != (R)0) ? voff : OOB;\n";
        }
        o << "  const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)x - "
          << shift << "ll), (short)0, " << (P.D * SZ + shift) << ", 0x00020000);\n"
          << "  const __amdgpu_buffer_rsrc_t ys = __builtin_amdgcn_make_buffer_rsrc((void*)((char*)y - "
          << shift << "ll), (short)0, " << (P.D * SZ + shift) << ", 0x00020000);\n";
        if (use_lds) o << "  const unsigned widx = act ? " << pad << "u + r : " << rows_lds - 1 << "u;\n";
        if (use_lds) o << "  __syncthreads();\n";
        o << "  const unsigned G = gridDim.x, b = blockIdx.x;\n"
          << "  const unsigned v = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;\n"
          << "  unsigned par = 0u;\n"
          << "  for (unsigned t = v; t < " << n_tiles << "u; t += G) {\n";
        for (int i : used_sites)
            if (!inner(i))
                o << "    const unsigned n" << i << " = (t / " << (P.M[i] / T_in) << "u) % " << P.d[i] << "u;\n";
        o << "    const unsigned F0 = t * " << T_in << "u;\n"
          << "    const C xf = LD(xs, voff, F0 * " << SZ << "u + " << shift << "u);\n";

        auto soff = [&](int64_t delta) {
            std::ostringstream s;
            s << "(F0 - " << static_cast<uint32_t>(static_cast<uint64_t>(delta)) << "u) * " << SZ << "u + " << shift
              << "u";
            return s.str();
        };
        auto ucond = [&](int c) -> std::string {  // uniform admissibility of the outer sites of channel c
            const auto& ch = P.chans[c];
            std::string cnd;
            auto add = [&](int site, int op) {
                if (inner(site)) return;
                const std::string e = adm_expr(p, site, op);
                if (!e.empty()) cnd = cnd.empty() ? e : cnd + " && " + e;
            };
            add(ch.a, ch.opa);
            if (ch.b >= 0) add(ch.b, ch.opb);
            return cnd.empty() ? "true" : cnd;
        };
        // outer and mixed channels read x through the buffer; every load is issued (out-of-range
        // offsets return 0 without a memory access), so the loads pipeline; groups of GS loads are
        // issued one group ahead of their use
        std::vector<int> cG = cO;
        cG.insert(cG.end(), cM.begin(), cM.end());
        const int GS = f32 ? 12 : 8;
        const int ng = static_cast<int>((cG.size() + GS - 1) / GS);
        auto emit_loads = [&](int g) {
            for (int i = g * GS; i < std::min<int>(cG.size(), (g + 1) * GS); ++i) {
                const int c = cG[i];
                const bool mixed = cls(P.chans[c].a, P.chans[c].b) == 2;
                const std::string base = mixed ? "vo" + std::to_string(c) : "voff";
                const std::string uc = ucond(c);
                o << "    const C s" << c << " = LD(xs, " << (uc == "true" ? base : "(" + uc + ") ? " + base + " : OOB")
                  << ", " << soff(P.chans[c].delta) << ");\n";
            }
        };
        auto emit_accum = [&](int g) {
            for (int i = g * GS; i < std::min<int>(cG.size(), (g + 1) * GS); ++i) {
                const int c = cG[i];
                const auto& ch = P.chans[c];
                const std::string cs = std::to_string(c), sc = "s" + cs;
                std::string f;
                if (cls(ch.a, ch.b) == 1)
                    f = ch.b >= 0 ? fac_uni2(ch.a, ch.opa, ch.b, ch.opb) : fac_uni(ch.a, ch.opa);
                else {
                    const bool ia = inner(ch.a);
                    f = fac_uni(ia ? ch.b : ch.a, ia ? ch.opb : ch.opa) + " * f" + cs;
                }
                o << "    { const R f = " << f << "; const R kr = cw" << cs << "r * f; ar += kr * " << sc
                  << ".x; ai += kr * " << sc << ".y;";
                if (complex_w)
                    o << " const R ki = cw" << cs << "i * f; ar -= ki * " << sc << ".y; ai += ki * " << sc << ".x;";
                o << " }\n";
            }
        };
        if (ng > 0) emit_loads(0);
        // diagonal weight for this tile
        o << "    R dr = dIr, di = dIi;\n";
        for (int g = 0; g < ndg; ++g) {
            const auto& dg = P.diags[g];
            const int k = cls(dg.a, dg.b);
            if (k == 0) continue;
            std::string f;
            if (k == 1) {
                f = dg.b >= 0 ? fac_uni2(dg.a, dg.opa, dg.b, dg.opb) : fac_uni(dg.a, dg.opa);
            } else {
                const bool ia = inner(dg.a);
                f = fac_uni(ia ? dg.b : dg.a, ia ? dg.opb : dg.opa) + " * fz" + std::to_string(g);
            }
            o << "    { const R f = " << f << "; dr += dw" << g << "r * f;";
            if (complex_w) o << " di += dw" << g << "i * f;";
            o << " }\n";
        }
        o << "    R ar = dr * xf.x - di * xf.y, ai = dr * xf.y + di * xf.x;\n";
        if (use_lds) {
            o << "    C* lb = lds + par * " << rows_lds << "u;\n"
              << "    lb[widx] = xf;\n"
              << "    __syncthreads();\n";
            for (int c : cI) {
                const std::string cs = std::to_string(c);
                const int64_t off = pad - P.chans[c].delta;
                o << "    { const C s = lb[r + " << off << "u]; ar += k" << cs << "r * s.x; ai += k" << cs << "r * s.y;";
                if (complex_w) o << " ar -= k" << cs << "i * s.y; ai += k" << cs << "i * s.x;";
                o << " }\n";
            }
            o << "    par ^= 1u;\n";
        }
        for (int g = 0; g < ng; ++g) {
            if (g + 1 < ng) emit_loads(g + 1);
            emit_accum(g);
        }
        o << "    { C out; out.x = ar; out.y = ai; ST(out, ys, voff, F0 * " << SZ << "u + " << shift << "u); }\n"
          << "  }\n}\n";

        std::ostringstream full;
        full << "// generated: " << P.N << " sites, " << nch << " channels (" << cI.size() << " inner, " << cM.size()
             << " mixed, " << cO.size() << " outer), " << ndg << " diagonal terms, inner block of " << T_in
             << " rows (sites " << k_in << ".." << P.N - 1 << ")\n";
        if (f32)
            full << "typedef float R;\ntypedef float C __attribute__((ext_vector_type(2)));\n"
                 << "#define LD(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64((rs), (int)(vo), (int)(so), 0))\n"
                 << "typedef unsigned U __attribute__((ext_vector_type(2)));\n"
                 << "#define ST(v, rs, vo, so) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, (v)), (rs), (int)(vo), (int)(so), 2)\n";
        else
            full << "typedef double R;\ntypedef double C __attribute__((ext_vector_type(2)));\n"
                 << "#define LD(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128((rs), (int)(vo), (int)(so), 0))\n"
                 << "typedef unsigned U __attribute__((ext_vector_type(4)));\n"
                 << "#define ST(v, rs, vo, so) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, (v)), (rs), (int)(vo), (int)(so), 2)\n";
        const std::string body = o.str();
        if (!pool.empty()) {
            full << "__constant__ R K[" << pool.size() << "] = {";
            for (size_t i = 0; i < pool.size(); ++i) full << (i ? ", " : "") << lit(pool[i], f32);
            full << "};\n";
        }
        full << pre.str() << body;
        return full.str();
    }
};

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Inner block: the low sites whose product T_in <= 1024 rows, preferring blocks of at least 256
// rows that fill whole wavefronts.
bool choose_tiling(const mrmf_plan_t* p, int inner_pref, int* k_in, int* T_in) {
    const int N = p->N;
    if (inner_pref > 0) {
        if (inner_pref > N) return false;
        int64_t T = 1;
        for (int i = N - inner_pref; i < N; ++i) T *= p->d[i];
        if (T > 1024) return false;
        *k_in = N - inner_pref;
        *T_in = static_cast<int>(T);
        return true;
    }
    double best = -1.0;
    int64_t T = 1;
    for (int k = N - 1; k >= 0; --k) {
        T *= p->d[k];
        if (T > 1024) break;
        const double eff = double(T) / double(round_up(T, 64));
        const double score = eff * std::min(1.0, double(T) / 256.0);
        if (score > best + 1e-12) {
            best = score;
            *k_in = k;
            *T_in = static_cast<int>(T);
        }
    }
    return best > 0.0;
}

}  // namespace

std::string spec_source(const mrmf_plan_t* p, int dtype, int* k_in_out, int* T_in_out) {
    const bool f32 = dtype == MRMF_DTYPE_C;
    const int64_t SZ = f32 ? 8 : 16;
    int k_in = 0, T_in = 0;
    if (!choose_tiling(p, p->inner_pref, &k_in, &T_in)) return "";
    const int64_t n_tiles = p->D / T_in;
    if (p->D * SZ + int64_t(T_in) * SZ >= (int64_t(1) << 31) || n_tiles >= (int64_t(1) << 31)) return "";
    Gen gen{p, f32, k_in, T_in, static_cast<int>(round_up(T_in, 64)), n_tiles};
    *k_in_out = k_in;
    *T_in_out = T_in;
    return gen.source();
}

namespace {

mrmf_status compile_spec(mrmf_plan_t* p, int dtype, SpecKernel& K) {
    K.tried = true;
    K.ok = false;
    int k_in = 0, T_in = 0;
    const std::string src = spec_source(p, dtype, &k_in, &T_in);
    if (src.empty()) {
        K.log = "plan does not qualify for the specialized kernel";
        return MRMF_E_UNSUPPORTED;
    }
    const int64_t n_tiles = p->D / T_in;
    const int block = static_cast<int>(round_up(T_in, 64));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MRMF_E_HIP;
    std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mrmf_spec.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return MRMF_E_HIP;
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult cr = hiprtcCompileProgram(prog, 7, opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string log(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &log[0]);
    if (cr != HIPRTC_SUCCESS) {
        K.log = "hiprtc: " + log + "\n" + src;
        hiprtcDestroyProgram(&prog);
        return MRMF_E_UNSUPPORTED;
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    std::vector<char> code(code_size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    hipModule_t mod;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess) return MRMF_E_HIP;
    hipFunction_t fn;
    if (hipModuleGetFunction(&fn, mod, "mrmf_spec") != hipSuccess) {
        hipModuleUnload(mod);
        return MRMF_E_HIP;
    }
    int per_cu = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t grid = int64_t(per_cu) * prop.multiProcessorCount;
    if (grid > n_tiles) grid = n_tiles;
    if (grid >= 8) grid -= grid % 8;
    K.mod = mod;
    K.fn = fn;
    K.k_in = k_in;
    K.T_in = T_in;
    K.block = block;
    K.grid = static_cast<int32_t>(grid);
    K.n_tiles = n_tiles;
    K.device = dev;
    K.log = src;
    K.ok = true;
    return MRMF_OK;
}

}  // namespace

mrmf_status spec_prepare(mrmf_plan_t* p, int dtype) {
    if (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C) return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mtx);
    SpecKernel& K = p->spec[dtype];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    if (K.tried && K.device == dev) return K.ok ? MRMF_OK : MRMF_E_UNSUPPORTED;
    if (K.mod) hipModuleUnload(K.mod);
    K = SpecKernel{};
    K.device = dev;
    return compile_spec(p, dtype, K);
}

mrmf_status spec_launch(mrmf_plan_t* p, int dtype, const void* theta, const void* x, void* y, hipStream_t s,
                        const int32_t* d_skip) {
    mrmf_status st = spec_prepare(p, dtype);
    if (st != MRMF_OK) return st;
    const SpecKernel& K = p->spec[dtype];
    struct {
        const void* theta;
        const void* x;
        void* y;
        const int32_t* skip;
    } args{theta, x, y, d_skip};
    size_t size = sizeof(args);
    void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size, HIP_LAUNCH_PARAM_END};
    return hip_status(hipModuleLaunchKernel(K.fn, K.grid, 1, 1, K.block, 1, 1, 0, s, nullptr, config));
}

}  // namespace mrmf

mrmf_plan_t::~mrmf_plan_t() {
    for (auto& k : spec)
        if (k.mod) hipModuleUnload(k.mod);
}

extern "C" {

mrmf_status mrmf_plan_set_kernel(mrmf_plan plan, int32_t kind, int32_t inner_sites) {
    if (!plan || kind < MRMF_KERNEL_AUTO || kind > MRMF_KERNEL_SPECIALIZED || inner_sites < 0 ||
        inner_sites > plan->N)
        return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mtx);
    plan->kernel_mode = kind;
    if (plan->inner_pref != inner_sites) {
        plan->inner_pref = inner_sites;
        for (auto& k : plan->spec) {
            if (k.mod) hipModuleUnload(k.mod);
            k = mrmf::SpecKernel{};
        }
    }
    return MRMF_OK;
}

mrmf_status mrmf_plan_prepare(mrmf_plan plan, int32_t dtype) {
    if (!plan || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C)) return MRMF_E_INVALID_ARG;
    if (plan->kernel_mode == MRMF_KERNEL_GENERIC) return MRMF_OK;
    const mrmf_status st = mrmf::spec_prepare(plan, dtype);
    if (st == MRMF_E_UNSUPPORTED && plan->kernel_mode == MRMF_KERNEL_AUTO) return MRMF_OK;
    return st;
}

mrmf_status mrmf_plan_kernel_source(mrmf_plan plan, int32_t dtype, char* buf, size_t cap, size_t* len) {
    if (!plan || !len || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C) || (cap > 0 && !buf))
        return MRMF_E_INVALID_ARG;
    int k_in = 0, T_in = 0;
    const std::string src = mrmf::spec_source(plan, dtype, &k_in, &T_in);
    if (src.empty()) return MRMF_E_UNSUPPORTED;
    *len = src.size();
    if (cap > 0) {
        const size_t n = src.size() < cap - 1 ? src.size() : cap - 1;
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
    }
    return MRMF_OK;
}

mrmf_status mrmf_plan_kernel_info(mrmf_plan plan, int32_t dtype, int32_t* out) {
    if (!plan || !out || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C)) return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mtx);
    const mrmf::SpecKernel& K = plan->spec[dtype];
    const bool spec = plan->kernel_mode != MRMF_KERNEL_GENERIC && K.ok;
    out[0] = spec ? MRMF_KERNEL_SPECIALIZED : MRMF_KERNEL_GENERIC;
    out[1] = spec ? plan->N - K.k_in : 0;
    out[2] = spec ? K.T_in : 0;
    out[3] = spec ? K.block : 256;
    out[4] = spec ? K.grid : 0;
    out[5] = spec ? static_cast<int32_t>(K.n_tiles) : 0;
    return MRMF_OK;
}

}  // extern "C"
