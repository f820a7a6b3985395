// Plan-specialized matvec kernels, generated as HIP source and compiled with hiprtc for the current
// device.  The generated kernel applies the same map as the generic one (target-driven gather, Sec. II;
// digits by Eq. decode; channels by Eqs. src_digit_two_site / sourceoffset; ladder factors of App. A,
// App. B, App. C) with the plan's structure baked in.
//
// Index space.  The sites split into three groups, most significant first:
//   uniform  [0, k_u)     digits fixed for a whole super-tile (scalar registers)
//   unrolled [k_u, k_in)  P_U digit combinations handled by every thread, one unrolled copy each, so
//                         these digits are compile-time constants inside a copy
//   inner    [k_in, N)    T_in rows, one per thread
// A super-tile is the P_U * T_in consecutive rows sharing the uniform digits.  Optionally site 0 is
// unrolled as well: a super-tile is then d_0 such runs of P_C * T_in rows, M_0 rows apart, so terms
// between site 0 and the unrolled/inner sites (the closing bond of a ring) become static.  Persistent blocks sweep
// the super-tiles; tiles are dealt so that the 8 XCDs each work on a contiguous stretch at a time.
//
// Terms.  A term touching only unrolled/inner sites is "static": its coefficient per thread and copy is
// fixed for the whole kernel (registers) and its source row lies inside the super-tile, whose x is staged
// in LDS (zeroed halo rows absorb inadmissible lanes, whose coefficient is 0).  A term touching only
// uniform sites is "uniform"; one touching both is "mixed".  Their uniform parts (theta-weighted ladder
// factors) are computed once per super-tile by a few lanes into an LDS table; their admissibility is
// decided on the scalar unit, and an inadmissible load gets an out-of-range buffer offset (no memory
// access, value 0), so every load is issued unconditionally and the loads pipeline.  y is written with
// non-temporal buffer stores.
#include <hip/hiprtc.h>

#include <array>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <sstream>
#include <tuple>

#include "mrmf_internal.h"

namespace mrmf {
namespace {

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

std::string lit(double v, bool f32) {
    char buf[64];
    if (f32)
        std::snprintf(buf, sizeof buf, "%af", static_cast<double>(static_cast<float>(v)));
    else
        std::snprintf(buf, sizeof buf, "%a", v);
    return buf;
}

std::string ulit(uint64_t v) {
    char buf[32];
    std::snprintf(buf, sizeof buf, "%" PRIu64 "ull", v);
    return buf;
}

// Factor <n|O|n - q> of a local operator at target digit n, 0 where the source digit is outside 0..d-1.
std::vector<double> factor_table(const mrmf_plan_t* p, int site, int op) {
    const int d = p->d[site], tab = p->tab[site];
    std::vector<double> t(d, 0.0);
    for (int n = 0; n < d; ++n) t[n] = local_factor_host(p, site, op, n);
    return t;
}

// ceil(2^64 / d): floor(n / d) = hi64(magic * n) for every n < 2^32
uint64_t magic_of(uint64_t d) { return d <= 1 ? 0 : ~uint64_t(0) / d + 1; }

struct Gen {
    const mrmf_plan_t* p;
    bool f32;
    Tile tl;
    int block;
    int64_t n_st;
    int sched = 0;       // MRMF_SCHED_*
    bool bskip = false;  // skip a channel whose uniform digits are inadmissible with a scalar branch
    int gs = 0;          // channels per load group (0: default)
    int variant = 0;     // MRMF_VARIANT_*
    // 64-bit addressing: the super-tile base is a 64-bit byte offset and every access builds its buffer
    // resource at base + scalar offset (a single resource with 32-bit offsets covers 2 GiB only)
    bool wide = false;
    // Chebyshev-step epilogue (time propagation): instead of y = H x the kernel computes
    // p = ea (H x) + eb x + eg y, writes it to y and adds (ecr + i eci) p to acc
    bool epi = false;
    int waves_per_eu = 0;  // > 0: ask the compiler for at least this many waves per SIMD (register budget)
    int far_nt = 0;        // > 0: gathers reaching |Delta| >= 2^far_nt bytes use LDN (non-temporal)
    int far_dir = 0;       // which of them: 0 both directions, 1 sources behind (Delta > 0), 2 ahead
    int outer_first = 0;   // the k most significant (uniform) sites vary fastest in the sweep

    std::string kernel_head() const {
        std::ostringstream o;
        o << "extern \"C\" __global__ __launch_bounds__(" << block << ") ";
        if (waves_per_eu > 0) o << "__attribute__((amdgpu_waves_per_eu(" << waves_per_eu << "))) ";
        o << "void " << (epi ? "mrmf_spec_cheb" : "mrmf_spec")
          << "(const R* __restrict__ theta,\n    const C* __restrict__ x, C* __restrict__ y, ";
        if (epi) o << "C* __restrict__ acc, R ea, R eb, R eg, R ecr, R eci, ";
        o << "const int* __restrict__ skip) {\n  if (skip != nullptr && *skip != 0) return;\n";
        return o.str();
    }
    // store of copy j's result out (= (H x) at the row) at scalar offset so; xj is the row's own x
    std::string store_out(const std::string& ind, int64_t j, const std::string& so, bool braces) const {
        std::ostringstream o;
        const std::string J = std::to_string(j);
        if (!epi) {
            o << ind << (braces ? "{ " : "") << "C out; out.x = a" << J << "r; out.y = a" << J << "i; ST(out, ys, voff, "
              << so << ");" << (braces ? " }" : "") << "\n";
            return o.str();
        }
        // the scheduling barrier keeps the two extra loads next to their use (hoisted over the whole
        // super-tile they would hold two vectors of registers per unrolled copy)
        o << ind << "{ __builtin_amdgcn_sched_barrier(0);\n"
          << ind << "  const C pv = LD(ys, voff, " << so << "), av = LD(as, voff, " << so << ");\n"
          << ind << "  C np; np.x = ea * a" << J << "r + eb * x" << J << ".x + eg * pv.x; np.y = ea * a" << J << "i + eb * x"
          << J << ".y + eg * pv.y;\n"
          << ind << "  ST(np, ys, voff, " << so << ");\n"
          << ind << "  C na; na.x = av.x + ecr * np.x - eci * np.y; na.y = av.y + ecr * np.y + eci * np.x;\n"
          << ind << "  ST(na, as, voff, " << so << "); }\n";
        return o.str();
    }

    // scalar byte offset of copy j's rows shifted by -delta, relative to a super-tile base `b`
    std::string soff_expr(const std::string& b, int64_t j, int64_t delta) const {
        const int64_t sz = SZ();
        std::ostringstream s;
        if (wide)
            s << b << " + (unsigned long long)(" << (copy_off(j) * sz - delta * sz) << "ll)";
        else
            s << b << " + " << static_cast<uint32_t>(static_cast<uint64_t>(copy_off(j) * sz - delta * sz)) << "u";
        return s.str();
    }
    // row offset of unrolled copy j from its super-tile base
    int64_t copy_off(int64_t j) const {
        int64_t off = (j % tl.P_C) * tl.T_in;
        for (int s = 0; s < tl.n_top; ++s) off += udigit(s, j) * p->M[s];
        return off;
    }
    // Delta of a static channel in the LDS layout, where copy j sits at j * T_in: the unrolled site 0 moves
    // by P_C * T_in rows there instead of M_0
    int64_t lds_delta(int c) const {
        const auto& ch = p->chans[c];
        int64_t d = ch.delta;
        if (is_top(ch.a)) d += int64_t(ch.qa) * (cstride(ch.a) * tl.T_in - p->M[ch.a]);
        if (is_top(ch.b)) d += int64_t(ch.qb) * (cstride(ch.b) * tl.T_in - p->M[ch.b]);
        return d;
    }
    // declaration of the super-tile base `b` for super-tile `t` (shift: the 32-bit form's base offset)
    // Natural super-tile index of sweep position e.  With outer_first = k the sweep visits the P_k
    // combinations of the k most significant sites back to back (their channels then read super-tiles
    // that neighbouring blocks of the same XCD load at the same time) and the rest in natural order.
    std::string tmap(const std::string& e) const {
        int64_t pk = 1;
        for (int s = tl.n_top > 0 ? tl.k_u : 0; s < std::min(outer_first, tl.k_u); ++s) pk *= p->d[s];
        if (pk <= 1) return e;
        return "((" + e + ") % " + std::to_string(pk) + "u * " + std::to_string(n_st / pk) + "u + (" + e + ") / " +
               std::to_string(pk) + "u)";
    }
    std::string base_decl(const std::string& b, const std::string& t, int64_t shift) const {
        std::ostringstream s;
        if (wide)
            s << "const unsigned long long " << b << " = (unsigned long long)(" << t << ") * " << STC() * SZ() << "ull;";
        else
            s << "const unsigned " << b << " = " << (t.find(' ') != std::string::npos ? "(" + t + ")" : t) << " * "
              << STC() * SZ() << "u + " << shift << "u;";
        return s.str();
    }
    std::string rsrc_decls(int64_t shift, int64_t nrec) const {
        std::ostringstream o;
        if (wide) {
            o << "  const char* const xs = (const char*)x;\n  char* const ys = (char*)y;\n";
            if (epi) o << "  char* const as = (char*)acc;\n";
        } else {
            o << "  const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)x - " << shift
              << "ll), (short)0, " << nrec << ", 0x00020000);\n"
              << "  const __amdgpu_buffer_rsrc_t ys = __builtin_amdgcn_make_buffer_rsrc((void*)((char*)y - " << shift
              << "ll), (short)0, " << nrec << ", 0x00020000);\n";
            if (epi)
                o << "  const __amdgpu_buffer_rsrc_t as = __builtin_amdgcn_make_buffer_rsrc((void*)((char*)acc - " << shift
                  << "ll), (short)0, " << nrec << ", 0x00020000);\n";
        }
        return o.str();
    }
    // element types and the load / store macros LD(resource, lane offset, scalar offset), ST(value, ...)
    std::string prelude() const {
        std::ostringstream full;
        if (f32)
            full << "typedef float R;\ntypedef float C __attribute__((ext_vector_type(2)));\n"
                 << "typedef unsigned U __attribute__((ext_vector_type(2)));\n";
        else
            full << "typedef double R;\ntypedef double C __attribute__((ext_vector_type(2)));\n"
                 << "typedef unsigned U __attribute__((ext_vector_type(4)));\n";
        if (wide) {
            // a buffer resource per access, based at the super-tile's byte offset (scalar arithmetic only);
            // the lane offset stays a 32-bit register and a masked lane's 0x80000000 reads zero / drops
            // its store as in the 32-bit form
            const char* bits = f32 ? "64" : "128";
            full << "#define RS(p) __builtin_amdgcn_make_buffer_rsrc((void*)(p), (short)0, 0x7fffffff, 0x00020000)\n"
                 << "#define LD(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b" << bits
                 << "(RS((rs) + (so)), (int)(vo), 0, 0))\n"
                 << "#define LDN(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b" << bits
                 << "(RS((rs) + (so)), (int)(vo), 0, 2))\n"
                 << "#define ST(v, rs, vo, so) __builtin_amdgcn_raw_buffer_store_b" << bits
                 << "(__builtin_bit_cast(U, (v)), RS((rs) + (so)), (int)(vo), 0, 2)\n";
        } else if (f32) {
            full << "#define LD(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64((rs), (int)(vo), (int)(so), 0))\n"
                 << "#define LDN(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64((rs), (int)(vo), (int)(so), 2))\n"
                 << "#define ST(v, rs, vo, so) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, (v)), (rs), (int)(vo), (int)(so), 2)\n";
        } else {
            full << "#define LD(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128((rs), (int)(vo), (int)(so), 0))\n"
                 << "#define LDN(rs, vo, so) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128((rs), (int)(vo), (int)(so), 2))\n"
                 // 128-bit store: the offset goes into the VGPR operand and the scalar offset is the
                 // constant 0; with a register scalar offset the compiler inserts no wait state between
                 // the store and a following VALU write of its data registers, and the stored value was
                 // then observed to be overwritten
                 << "#define ST(v, rs, vo, so) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, (v)), (rs), (int)((unsigned)(vo) + (unsigned)(so)), 0, 2)\n";
        }
        return full.str();
    }

    int SZ() const { return f32 ? 8 : 16; }
    // a channel whose offset reaches far enough for a non-temporal load (MRMF_TUNE_FAR_LOADS)
    bool far(int64_t delta) const {
        if (far_nt <= 0 || (far_dir == 1 && delta <= 0) || (far_dir == 2 && delta >= 0)) return false;
        return static_cast<double>(delta < 0 ? -delta : delta) * SZ() >= std::ldexp(1.0, far_nt);
    }
    int op_shift(int op) const {
        if (op >= MRMF_OP_LOCAL_BASE) return p->lshift[op - MRMF_OP_LOCAL_BASE];
        switch (op) {
            case MRMF_OP_RAISE: return 1;
            case MRMF_OP_LOWER: return -1;
            case MRMF_OP_RAISE2: return 2;
            case MRMF_OP_LOWER2: return -2;
            default: return 0;
        }
    }
    bool is_inner(int s) const { return s >= tl.k_in; }
    bool is_top(int s) const { return s >= 0 && s < tl.n_top; }
    bool is_unrolled(int s) const { return (s >= tl.k_u && s < tl.k_in) || is_top(s); }
    bool is_static(int s) const { return s >= tl.k_u || is_top(s); }
    // copy-index stride of unrolled top site s (< n_top): the contiguous combinations vary fastest, then
    // sites n_top - 1 .. 0
    int64_t cstride(int s) const {
        int64_t c = tl.P_C;
        for (int u = s + 1; u < tl.n_top; ++u) c *= p->d[u];
        return c;
    }
    int64_t ST() const { return tl.T_in * tl.P_U; }   // rows of a super-tile (its LDS image)
    int64_t STC() const { return tl.T_in * tl.P_C; }  // stride of the super-tile bases in rows
    int udigit(int s, int64_t j) const {
        if (is_top(s)) return static_cast<int>((j / cstride(s)) % p->d[s]);
        return static_cast<int>(((j % tl.P_C) / (p->M[s] / tl.T_in)) % p->d[s]);
    }
    int kind(int a, int b) const {  // 0 static, 1 uniform, 2 mixed
        const bool sa = is_static(a);
        if (b < 0) return sa ? 0 : 1;
        const bool sb = is_static(b);
        if (sa && sb) return 0;
        if (!sa && !sb) return 1;
        return 2;
    }
    bool has_inner(int a, int b) const { return is_inner(a) || (b >= 0 && is_inner(b)); }
    bool has_unrolled(int a, int b) const { return is_unrolled(a) || (b >= 0 && is_unrolled(b)); }

    // constant pool (factor tables), shared by every lookup
    std::vector<double> pool;
    std::map<std::string, size_t> pool_index;
    size_t pool_add(const std::string& key, const std::vector<double>& t) {
        auto it = pool_index.find(key);
        if (it != pool_index.end()) return it->second;
        const size_t off = pool.size();
        pool.insert(pool.end(), t.begin(), t.end());
        pool_index[key] = off;
        return off;
    }
    size_t ftab(int s, int op) { return pool_add("F" + std::to_string(s) + "_" + std::to_string(op), factor_table(p, s, op)); }

    // per-lane factor of an inner site (select chain for small d, pool lookup otherwise)
    std::string lane_fac(int s, int op) {
        const std::vector<double> t = factor_table(p, s, op);
        const std::string n = "n" + std::to_string(s);
        const int d = static_cast<int>(t.size());
        if (d <= 4) {
            std::string e = lit(t[d - 1], f32);
            for (int i = d - 2; i >= 0; --i)
                e = "(" + n + " == " + std::to_string(i) + "u ? " + lit(t[i], f32) + " : " + e + ")";
            return e;
        }
        return "K[" + std::to_string(ftab(s, op)) + "u + " + n + "]";
    }
    // static part of a term in copy j: compile-time factor of unrolled sites and lane expression
    std::pair<double, std::string> static_part(int a, int opa, int b, int opb, int64_t j) {
        double c = 1.0;
        std::string e;
        auto add = [&](int s, int op) {
            if (s < 0 || !is_static(s)) return;
            if (is_unrolled(s)) {
                c *= factor_table(p, s, op)[udigit(s, j)];
            } else {
                const std::string f = lane_fac(s, op);
                e = e.empty() ? f : e + " * " + f;
            }
        };
        add(a, opa);
        add(b, opb);
        return {c, e};
    }
    std::string admit_uniform(int a, int opa, int b, int opb) const {
        std::string c;
        auto add = [&](int s, int op) {
            if (s < 0 || is_static(s)) return;
            // the source digit n - q must lie in 0..d-1 (q: the operator's digit shift)
            std::string e;
            const int q = op_shift(op), d = p->d[s];
            if (q >= d || d - 1 + q < 0)  // (S_+-)^2 on a spin 1/2: never admissible
                e = "false";
            else if (q > 0)
                e = "n" + std::to_string(s) + " >= " + std::to_string(q) + "u";
            else if (q < 0)
                e = "n" + std::to_string(s) + " <= " + std::to_string(d - 1 + q) + "u";
            if (!e.empty()) c = c.empty() ? e : c + " && " + e;
        };
        add(a, opa);
        add(b, opb);
        return c.empty() ? "true" : c;
    }

    // The masked form computes each tile-uniform coefficient on one lane of the first waves, so its
    // items (uniform and mixed channels, mixed diagonal terms) and its summed uniform diagonal terms
    // must each fit in the block.
    bool masked_fits() const {
        int nit = 0, nsum = 0;
        for (const auto& c : p->chans) nit += kind(c.a, c.b) != 0;
        for (const auto& g : p->diags) {
            const int k = kind(g.a, g.b);
            nit += k == 2;
            nsum += k == 1;
        }
        return nit <= block && nsum <= block;
    }

    std::string source() {
        const mrmf_plan_t& P = *p;
        const int sz = SZ();
        const int nch = static_cast<int>(P.chans.size()), ndg = static_cast<int>(P.diags.size());
        const int64_t T = tl.T_in, PU = tl.P_U, st = ST();
        bool cplx = false;
        for (const auto& c : P.chans) cplx |= c.wi != 0.0;
        for (const auto& g : P.diags) cplx |= g.wi != 0.0;

        std::vector<int> cS, cU, cM, gS, gU, gM;
        for (int c = 0; c < nch; ++c) {
            const int k = kind(P.chans[c].a, P.chans[c].b);
            (k == 0 ? cS : k == 1 ? cU : cM).push_back(c);
        }
        for (int g = 0; g < ndg; ++g) {
            const int k = kind(P.diags[g].a, P.diags[g].b);
            (k == 0 ? gS : k == 1 ? gU : gM).push_back(g);
        }
        int64_t dmax = 0, halo = 0;
        for (const auto& c : P.chans) dmax = std::max<int64_t>(dmax, c.delta);
        for (int c : cS) {  // inner part of Delta; the unrolled part moves between copies in the super-tile
            const auto& ch = P.chans[c];
            int64_t di = 0;
            if (is_inner(ch.a)) di += int64_t(ch.qa) * P.M[ch.a];
            if (ch.b >= 0 && is_inner(ch.b)) di += int64_t(ch.qb) * P.M[ch.b];
            halo = std::max<int64_t>(halo, di < 0 ? -di : di);
        }
        // buffer base shifted down by `shift` bytes so every scalar offset is non-negative
        const int64_t shift = (dmax + T) * sz;
        const int64_t nrec = (P.D + dmax + T) * sz;
        const bool use_lds = !cS.empty();
        const int64_t xrows = st + 2 * halo + 1;  // halo, super-tile, halo, one slot idle lanes write to
        const bool dbuf = use_lds && 2 * xrows * sz <= 49152;
        // uniform-part table items: uniform channels, mixed channels, mixed diagonal terms
        std::vector<std::pair<int, int>> items;
        for (int c : cU) items.push_back({0, c});
        for (int c : cM) items.push_back({0, c});
        for (int g : gM) items.push_back({1, g});
        const int nit = static_cast<int>(items.size()), nsum = static_cast<int>(gU.size());
        const int nw = block / 64;
        const int twaves = std::min(nw, std::max((nit + 63) / 64, (nsum + 63) / 64));
        std::map<int, int> item_of_chan, item_of_diag;
        for (int i = 0; i < nit; ++i) (items[i].first == 0 ? item_of_chan : item_of_diag)[items[i].second] = i;

        std::ostringstream pre, o;
        // per-item constants (global tables): for up to two uniform sites, the division magic of the
        // site multiplier counted in super-tiles, the dimension and its magic, the factor-table offset
        // (an absent site has quotient magic 1, so its digit is 0, dimension 1 and a 1.0 entry), the parameter
        // and the weight
        const size_t one = pool_add("ONE", {1.0});
        auto emit_items = [&](const std::string& pfx, const std::vector<std::tuple<int, int, int, int, int, double, double>>& its) {
            const int n = std::max<int>(1, its.size());
            std::ostringstream mam, da, dam, ta, mbm, db, dbm, tb, pr, wr, wi;
            for (size_t i = 0; i < its.size(); ++i) {
                std::vector<std::array<uint64_t, 3>> ss;  // (multiplier in super-tiles, d, table)
                for (auto so : {std::make_pair(std::get<0>(its[i]), std::get<1>(its[i])),
                                std::make_pair(std::get<2>(its[i]), std::get<3>(its[i]))}) {
                    if (so.first < 0 || is_static(so.first)) continue;
                    ss.push_back({static_cast<uint64_t>(P.M[so.first] / STC()), static_cast<uint64_t>(P.d[so.first]),
                                  static_cast<uint64_t>(ftab(so.first, so.second))});
                }
                // an absent site has multiplier 0: magic 1 makes its quotient, hence its digit, 0
                while (ss.size() < 2) ss.push_back({0, 1, static_cast<uint64_t>(one)});
                const char* sep = i ? ", " : "";
                mam << sep << ulit(ss[0][0] == 0 ? 1 : ss[0][0] == 1 ? 0 : magic_of(ss[0][0]));
                da << sep << ss[0][1] << "u";
                dam << sep << ulit(magic_of(ss[0][1]));
                ta << sep << ss[0][2] << "u";
                mbm << sep << ulit(ss[1][0] == 0 ? 1 : ss[1][0] == 1 ? 0 : magic_of(ss[1][0]));
                db << sep << ss[1][1] << "u";
                dbm << sep << ulit(magic_of(ss[1][1]));
                tb << sep << ss[1][2] << "u";
                pr << sep << std::get<4>(its[i]);
                wr << sep << lit(std::get<5>(its[i]), f32);
                wi << sep << lit(std::get<6>(its[i]), f32);
            }
            auto arr = [&](const char* ty, const char* nm, std::ostringstream& v) {
                const std::string s = v.str();
                pre << "__constant__ " << ty << " " << pfx << nm << "[" << n << "] = {" << (s.empty() ? "0" : s) << "};\n";
            };
            arr("unsigned long long", "mam", mam);
            arr("unsigned", "da", da);
            arr("unsigned long long", "dam", dam);
            arr("unsigned", "ta", ta);
            arr("unsigned long long", "mbm", mbm);
            arr("unsigned", "db", db);
            arr("unsigned long long", "dbm", dbm);
            arr("unsigned", "tb", tb);
            arr("int", "pr", pr);
            arr("R", "wr", wr);
            arr("R", "wi", wi);
        };
        if (twaves > 0) {
            std::vector<std::tuple<int, int, int, int, int, double, double>> its, sums;
            for (const auto& it : items) {
                if (it.first == 0) {
                    const auto& ch = P.chans[it.second];
                    its.emplace_back(ch.a, ch.opa, ch.b, ch.opb, ch.param, ch.wr, ch.wi);
                } else {
                    const auto& dg = P.diags[it.second];
                    its.emplace_back(dg.a, dg.opa, dg.b, dg.opb, dg.param, dg.wr, dg.wi);
                }
            }
            for (int g : gU) {
                const auto& dg = P.diags[g];
                sums.emplace_back(dg.a, dg.opa, dg.b, dg.opb, dg.param, dg.wr, dg.wi);
            }
            emit_items("I", its);
            emit_items("Q", sums);
        }

        o << "__device__ __forceinline__ unsigned dig(unsigned t, unsigned long long mm, unsigned d, unsigned long long dm) {\n"
          << "  const unsigned q = mm ? (unsigned)__umul64hi(mm, (unsigned long long)t) : t;\n"
          << "  return q - (unsigned)__umul64hi(dm, (unsigned long long)q) * d;\n}\n";
        o << kernel_head();
        if (use_lds) o << "  __shared__ C xl[" << (dbuf ? 2 : 1) * xrows << "];\n";
        if (nit > 0) {
            o << "  __shared__ R tr[2][" << nit << "];\n";
            if (cplx) o << "  __shared__ R ti[2][" << nit << "];\n";
        }
        if (nsum > 0) {
            o << "  __shared__ R dsr[2][" << twaves << "];\n";
            if (cplx) o << "  __shared__ R dsi[2][" << twaves << "];\n";
        }
        if (twaves > 0) o << "  __shared__ R Kl[KN_ALLOC];\n";  // the pool is complete only after codegen
        o << "  const unsigned tid = threadIdx.x;\n"
          << "  const bool act = tid < " << T << "u;\n"
          << "  const unsigned r = act ? tid : 0u;\n"
          << "  const unsigned OOB = 0x80000000u;\n"
          << "  const unsigned voff = act ? r * " << sz << "u : OOB;\n";
        if (use_lds) {
            o << "  for (unsigned i = tid; i < " << halo << "u; i += " << block << "u) {\n"
              << "    const C z = {(R)0, (R)0};\n";
            for (int b = 0; b < (dbuf ? 2 : 1); ++b)
                o << "    xl[" << b * xrows << "u + i] = z; xl[" << b * xrows + halo + st << "u + i] = z;\n";
            o << "  }\n";
            for (int64_t j = 0; j < PU; ++j)
                o << "  const unsigned w" << j << " = act ? " << halo + j * T << "u + r : " << xrows - 1 << "u;\n";
        }
        if (twaves > 0)
            o << "  for (unsigned i = tid; i < KN; i += " << block << "u) Kl[i] = K[i];\n";
        std::set<int> lane_sites, used_params;
        for (const auto& c : P.chans) {
            if (is_inner(c.a)) lane_sites.insert(c.a);
            if (c.b >= 0 && is_inner(c.b)) lane_sites.insert(c.b);
            used_params.insert(c.param);
        }
        for (const auto& g : P.diags) {
            if (is_inner(g.a)) lane_sites.insert(g.a);
            if (g.b >= 0 && is_inner(g.b)) lane_sites.insert(g.b);
            used_params.insert(g.param);
        }
        for (int s : lane_sites) o << "  const unsigned n" << s << " = (r / " << P.M[s] << "u) % " << P.d[s] << "u;\n";
        for (int q : used_params) o << "  const R th" << q << " = theta[" << q << "];\n";
        auto wexpr = [&](int param, double w) { return "th" + std::to_string(param) + " * " + lit(w, f32); };

        // static channel coefficients per copy (registers)
        std::map<std::pair<int, int64_t>, std::string> kS;
        for (int c : cS) {
            const auto& ch = P.chans[c];
            const bool unr = has_unrolled(ch.a, ch.b);
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(ch.a, ch.opa, ch.b, ch.opb, j);
                if (sp.first == 0.0) continue;
                if (!unr && j > 0 && kS.count({c, 0})) {
                    kS[{c, j}] = kS[{c, 0}];
                    continue;
                }
                const std::string nm = "k" + std::to_string(c) + "_" + std::to_string(j);
                const std::string le = sp.second.empty() ? std::string("(R)1") : sp.second;
                o << "  const R " << nm << "r = act ? " << wexpr(ch.param, ch.wr) << " * " << lit(sp.first, f32) << " * "
                  << le << " : (R)0;\n";
                if (cplx)
                    o << "  const R " << nm << "i = act ? " << wexpr(ch.param, ch.wi) << " * " << lit(sp.first, f32)
                      << " * " << le << " : (R)0;\n";
                kS[{c, j}] = nm;
            }
        }
        // mixed channels: static factor per copy; lane admissibility folded into the buffer offset
        std::map<std::pair<int, int64_t>, std::string> fM;
        for (int c : cM) {
            const auto& ch = P.chans[c];
            std::string lane_e;
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(ch.a, ch.opa, ch.b, ch.opb, j);
                if (sp.first == 0.0) continue;
                if (!sp.second.empty()) lane_e = sp.second;
                const std::string nm = "f" + std::to_string(c) + "_" + std::to_string(j);
                o << "  const R " << nm << " = " << lit(sp.first, f32) << " * " << (sp.second.empty() ? "(R)1" : sp.second)
                  << ";\n";
                fM[{c, j}] = nm;
            }
            if (has_inner(ch.a, ch.b) && !lane_e.empty())
                o << "  const unsigned vo" << c << " = (" << lane_e << " != (R)0) ? voff : OOB;\n";
        }
        // diagonal: static part per copy; static factor of mixed terms per copy
        for (int64_t j = 0; j < PU; ++j) {
            o << "  R dS" << j << "r = 0, dS" << j << "i = 0;\n";
            for (int g : gS) {
                const auto& dg = P.diags[g];
                const auto sp = static_part(dg.a, dg.opa, dg.b, dg.opb, j);
                if (sp.first == 0.0) continue;
                const std::string le = sp.second.empty() ? std::string("(R)1") : sp.second;
                o << "  { const R f = " << lit(sp.first, f32) << " * " << le << "; dS" << j << "r += "
                  << wexpr(dg.param, dg.wr) << " * f;";
                if (cplx) o << " dS" << j << "i += " << wexpr(dg.param, dg.wi) << " * f;";
                o << " }\n";
            }
        }
        std::map<std::pair<int, int64_t>, std::string> fD;
        for (int g : gM) {
            const auto& dg = P.diags[g];
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(dg.a, dg.opa, dg.b, dg.opb, j);
                if (sp.first == 0.0) continue;
                const std::string nm = "z" + std::to_string(g) + "_" + std::to_string(j);
                o << "  const R " << nm << " = " << lit(sp.first, f32) << " * " << (sp.second.empty() ? "(R)1" : sp.second)
                  << ";\n";
                fD[{g, j}] = nm;
            }
        }
        // table lanes: lane l of wave w owns item 64 w + l and uniform diagonal term 64 w + l
        if (twaves > 0) {
            o << "  const unsigned wv = tid >> 6, ln = tid & 63u, it = tid;\n"
              << "  const bool has_it = it < " << nit << "u, has_q = it < " << nsum << "u;\n"
              << "  const unsigned ii = has_it ? it : 0u, qq = has_q ? it : 0u;\n"
              << "  const unsigned long long i_mam = Imam[ii], i_dam = Idam[ii], i_mbm = Imbm[ii], i_dbm = Idbm[ii];\n"
              << "  const unsigned i_da = Ida[ii], i_db = Idb[ii], i_ta = Ita[ii], i_tb = Itb[ii];\n"
              << "  const R i_wr = theta[Ipr[ii]] * Iwr[ii], i_wi = theta[Ipr[ii]] * Iwi[ii];\n"
              << "  const unsigned long long q_mam = Qmam[qq], q_dam = Qdam[qq], q_mbm = Qmbm[qq], q_dbm = Qdbm[qq];\n"
              << "  const unsigned q_da = Qda[qq], q_db = Qdb[qq], q_ta = Qta[qq], q_tb = Qtb[qq];\n"
              << "  const R q_wr = has_q ? theta[Qpr[qq]] * Qwr[qq] : (R)0, q_wi = has_q ? theta[Qpr[qq]] * Qwi[qq] : (R)0;\n";
        }
        o << rsrc_decls(shift, nrec)
          << "  __syncthreads();\n"
          << "  const unsigned G = gridDim.x, b = blockIdx.x;\n"
          << "  unsigned par = 0u;\n";
        // loop over sweep positions; t is the natural super-tile index (the same unless outer_first > 0)
        const bool remap = tmap("ts") != "ts";
        const std::string tv = remap ? "ts" : "t";
        if (sched == MRMF_SCHED_XCD_CHUNK) {
            // XCD x (= b mod 8) sweeps the contiguous range [x C, (x + 1) C) of super-tiles with its G / 8
            // blocks side by side, so neighbouring super-tiles are read through the same L2
            o << "  const unsigned nx = (G % 8u == 0u) ? 8u : 1u, GX = G / nx, xcd = b % nx;\n"
              << "  const unsigned Cx = (" << n_st << "u + nx - 1u) / nx;\n"
              << "  const unsigned t_end = (xcd + 1u) * Cx < " << n_st << "u ? (xcd + 1u) * Cx : " << n_st << "u;\n"
              << "  for (unsigned " << tv << " = xcd * Cx + b / nx; " << tv << " < t_end; " << tv << " += GX) {\n";
        } else if (sched == MRMF_SCHED_BLOCK_RUN) {
            // every block sweeps its own contiguous run of super-tiles, so a neighbour read as a channel
            // source is read again, as the block's own rows, a few super-tiles later through its own L1;
            // the runs of the blocks of one XCD are adjacent
            o << "  const unsigned v = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;\n"
              << "  const unsigned t_end = (unsigned)(((unsigned long long)(v + 1u) * " << n_st << "ull) / G);\n"
              << "  for (unsigned " << tv << " = (unsigned)(((unsigned long long)v * " << n_st << "ull) / G); " << tv << " < t_end; ++" << tv << ") {\n";
        } else {
            // the grid sweeps windows of G consecutive super-tiles; XCD x takes the x-th eighth of each
            o << "  const unsigned v = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;\n"
              << "  for (unsigned " << tv << " = v; " << tv << " < " << n_st << "u; " << tv << " += G) {\n";
        }
        if (remap) o << "    const unsigned t = " << tmap("ts") << ";\n";
        std::set<int> uni_sites;
        for (const auto& c : P.chans) {
            if (!is_static(c.a)) uni_sites.insert(c.a);
            if (c.b >= 0 && !is_static(c.b)) uni_sites.insert(c.b);
        }
        for (int s : uni_sites) o << "    const unsigned n" << s << " = (t / " << P.M[s] / STC() << "u) % " << P.d[s] << "u;\n";
        o << "    " << base_decl("F0", "t", shift) << "\n";
        auto soff = [&](int64_t j, int64_t delta) { return soff_expr("F0", j, delta); };
        for (int64_t j = 0; j < PU; ++j) o << "    const C x" << j << " = LD(xs, voff, " << soff(j, 0) << ");\n";
        std::vector<int> cG = cU;
        cG.insert(cG.end(), cM.begin(), cM.end());
        for (int c : cG) {
            const auto& ch = P.chans[c];
            bool lane = false;
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(ch.a, ch.opa, ch.b, ch.opb, j);
                if (sp.first != 0.0 && !sp.second.empty()) lane = true;
            }
            const std::string base = (kind(ch.a, ch.b) == 2 && lane) ? "vo" + std::to_string(c) : "voff";
            const std::string ad = admit_uniform(ch.a, ch.opa, ch.b, ch.opb);
            if (bskip) {
                o << "    const bool q" << c << " = " << ad << ";\n";
                o << "    const unsigned u" << c << " = " << base << ";\n";
            } else {
                o << "    const unsigned u" << c << " = " << (ad == "true" ? base : "(" + ad + ") ? " + base + " : OOB") << ";\n";
            }
        }
        const int GS = gs > 0 ? gs : (f32 ? 10 : 6);  // channels per load group
        const int ngr = static_cast<int>((cG.size() + GS - 1) / GS);
        auto emit_loads = [&](int g) {
            for (int i = g * GS; i < std::min<int>(cG.size(), (g + 1) * GS); ++i) {
                const int c = cG[i];
                const auto& ch = P.chans[c];
                const char* ld = far(ch.delta) ? "LDN" : "LD";
                for (int64_t j = 0; j < PU; ++j) {
                    if (kind(ch.a, ch.b) == 2 && !fM.count({c, j})) continue;
                    if (bskip)
                        o << "    C s" << c << "_" << j << " = {(R)0, (R)0}; if (q" << c << ") s" << c << "_" << j
                          << " = " << ld << "(xs, u" << c << ", " << soff(j, ch.delta) << ");\n";
                    else
                        o << "    const C s" << c << "_" << j << " = " << ld << "(xs, u" << c << ", " << soff(j, ch.delta)
                          << ");\n";
                }
            }
        };
        if (ngr > 0) emit_loads(0);
        if (twaves > 0) {
            o << "    if (wv < " << twaves << "u) {\n"
              << "      if (has_it) {\n"
              << "        const unsigned na = dig(t, i_mam, i_da, i_dam), nb = dig(t, i_mbm, i_db, i_dbm);\n"
              << "        const R f = Kl[i_ta + na] * Kl[i_tb + nb];\n"
              << "        tr[par][ii] = i_wr * f;\n"
              << (cplx ? "        ti[par][ii] = i_wi * f;\n" : "")
              << "      }\n";
            if (nsum > 0) {
                o << "      const unsigned ma = dig(t, q_mam, q_da, q_dam), mb = dig(t, q_mbm, q_db, q_dbm);\n"
                  << "      const R g = Kl[q_ta + ma] * Kl[q_tb + mb];\n"
                  << "      R vr = q_wr * g, vi = q_wi * g;\n"
                  << "      for (int k = 32; k > 0; k >>= 1) { vr += __shfl_down(vr, k, 64);"
                  << (cplx ? " vi += __shfl_down(vi, k, 64);" : "") << " }\n"
                  << "      if (ln == 0u) { dsr[par][wv] = vr;" << (cplx ? " dsi[par][wv] = vi;" : "") << " }\n";
            }
            o << "    }\n";
        }
        if (use_lds) {
            o << "    C* lb = xl" << (dbuf ? " + par * " + std::to_string(xrows) + "u" : std::string("")) << ";\n";
            for (int64_t j = 0; j < PU; ++j) o << "    lb[w" << j << "] = x" << j << ";\n";
        }
        o << "    __syncthreads();\n"
          << "    R dUr = (R)0, dUi = (R)0;\n";
        for (int w = 0; w < (nsum > 0 ? twaves : 0); ++w)
            o << "    dUr += dsr[par][" << w << "];" << (cplx ? " dUi += dsi[par][" + std::to_string(w) + "];" : "") << "\n";
        for (int64_t j = 0; j < PU; ++j) {
            o << "    R a" << j << "r, a" << j << "i;\n    {\n      R dr = dS" << j << "r + dUr, di = dS" << j << "i + dUi;\n";
            for (int g : gM) {
                auto it = fD.find({g, j});
                if (it == fD.end()) continue;
                const int idx = item_of_diag[g];
                o << "      dr += tr[par][" << idx << "] * " << it->second << ";";
                if (cplx) o << " di += ti[par][" << idx << "] * " << it->second << ";";
                o << "\n";
            }
            o << "      a" << j << "r = dr * x" << j << ".x - di * x" << j << ".y; a" << j << "i = dr * x" << j
              << ".y + di * x" << j << ".x;\n    }\n";
        }
        auto acc = [&](int64_t j, const std::string& kr, const std::string& ki, const std::string& s) {
            o << "a" << j << "r += " << kr << " * " << s << ".x; a" << j << "i += " << kr << " * " << s << ".y;";
            if (!ki.empty())
                o << " a" << j << "r -= " << ki << " * " << s << ".y; a" << j << "i += " << ki << " * " << s << ".x;";
        };
        if (use_lds) {
            for (int c : cS) {
                for (int64_t j = 0; j < PU; ++j) {
                    auto it = kS.find({c, j});
                    if (it == kS.end()) continue;
                    const int64_t off = halo + j * T - lds_delta(c);
                    o << "    { const C s = lb[r + " << off << "u]; ";
                    acc(j, it->second + "r", cplx ? it->second + "i" : "", "s");
                    o << " }\n";
                }
            }
            if (!dbuf) o << "    __syncthreads();\n";
        }
        auto emit_accum = [&](int g) {
            for (int i = g * GS; i < std::min<int>(cG.size(), (g + 1) * GS); ++i) {
                const int c = cG[i];
                const auto& ch = P.chans[c];
                const int idx = item_of_chan[c];
                o << "    " << (bskip ? "if (q" + std::to_string(c) + ") " : std::string("")) << "{ const R kr = tr[par]["
                  << idx << "];" << (cplx ? " const R ki = ti[par][" + std::to_string(idx) + "];" : "") << "\n";
                for (int64_t j = 0; j < PU; ++j) {
                    const std::string s = "s" + std::to_string(c) + "_" + std::to_string(j);
                    if (kind(ch.a, ch.b) == 1) {
                        o << "      ";
                        acc(j, "kr", cplx ? "ki" : "", s);
                        o << "\n";
                    } else {
                        auto it = fM.find({c, j});
                        if (it == fM.end()) continue;
                        o << "      { const R mr = kr * " << it->second << ";"
                          << (cplx ? " const R mi = ki * " + it->second + ";" : "") << " ";
                        acc(j, "mr", cplx ? "mi" : "", s);
                        o << " }\n";
                    }
                }
                o << "    }\n";
            }
        };
        for (int g = 0; g < ngr; ++g) {
            if (g + 1 < ngr) emit_loads(g + 1);
            emit_accum(g);
        }
        for (int64_t j = 0; j < PU; ++j)
            o << store_out("    ", j, soff(j, 0), true);
        o << "    par ^= 1u;\n  }\n}\n";

        std::ostringstream full;
        full << "// generated: " << P.N << " sites, " << nch << " channels (" << cS.size() << " static, " << cM.size()
             << " mixed, " << cU.size() << " uniform), " << ndg << " diagonal terms; " << T
             << " rows per block (sites " << tl.k_in << ".." << P.N - 1 << "), " << PU << " unrolled copies (sites "
             << tl.k_u << ".." << tl.k_in - 1 << "), " << n_st << " super-tiles\n";
        full << prelude();
        full << "#define KN " << pool.size() << "u\n#define KN_ALLOC " << std::max<size_t>(pool.size(), 1) << "\n";
        full << "__constant__ R K[" << std::max<size_t>(pool.size(), 1) << "] = {";
        if (pool.empty()) full << "0";
        for (size_t i = 0; i < pool.size(); ++i) full << (i ? ", " : "") << lit(pool[i], f32);
        full << "};\n" << pre.str() << o.str();
        return full.str();
    }
    // Second form of the generated kernel.  Per super-tile, the channels that read outside it (uniform and
    // mixed) are not issued as masked loads: a few lanes evaluate their tile-uniform admissibility and
    // coefficient and append the admissible ones, per unrolled copy, to a compact list in LDS (ballot
    // and prefix count, so the order is deterministic); every thread then walks the list in chunks of U
    // entries, issuing U gathers before their U accumulations.  A mixed channel's per-row factor (its
    // inner-site part, zero where that digit is inadmissible) comes from a per-thread LDS table indexed by
    // the entry's group.  The self rows of the next super-tile are loaded before the current one is
    // computed.
    std::string source_v2() {
        const mrmf_plan_t& P = *p;
        const int sz = SZ();
        const int nch = static_cast<int>(P.chans.size()), ndg = static_cast<int>(P.diags.size());
        const int64_t T = tl.T_in, PU = tl.P_U, st = ST();
        bool cplx = false;
        for (const auto& c : P.chans) cplx |= c.wi != 0.0;
        for (const auto& g : P.diags) cplx |= g.wi != 0.0;
        std::vector<int> cS, cG, gS, gU, gM;
        for (int c = 0; c < nch; ++c) (kind(P.chans[c].a, P.chans[c].b) == 0 ? cS : cG).push_back(c);
        for (int g = 0; g < ndg; ++g) {
            const int k = kind(P.diags[g].a, P.diags[g].b);
            (k == 0 ? gS : k == 1 ? gU : gM).push_back(g);
        }
        int64_t dmax = 0, halo = 0;
        for (const auto& c : P.chans) dmax = std::max<int64_t>(dmax, c.delta);
        for (int c : cS) {
            const auto& ch = P.chans[c];
            int64_t di = 0;
            if (is_inner(ch.a)) di += int64_t(ch.qa) * P.M[ch.a];
            if (ch.b >= 0 && is_inner(ch.b)) di += int64_t(ch.qb) * P.M[ch.b];
            halo = std::max<int64_t>(halo, di < 0 ? -di : di);
        }
        const int64_t shift = (dmax + T) * sz;
        const int64_t nrec = (P.D + dmax + T) * sz;
        const bool use_lds = !cS.empty();
        const int64_t xrows = st + 2 * halo + 1;
        const int nw = block / 64;
        const int U = gs > 0 ? gs : (f32 ? 8 : 6);  // gathers issued per chunk of the list

        // lane groups: (inner site, operator) of a mixed channel's per-row factor; group 0 is 1.0, the
        // last group is the sentinel 0.0
        std::map<std::pair<int, int>, int> group_of;
        auto lane_group = [&](int a, int opa, int b, int opb) {
            int s = -1, op = 0;
            if (is_inner(a)) { s = a; op = opa; }
            if (b >= 0 && is_inner(b)) {
                if (s >= 0) return -2;  // both inner: only a static channel can have that
                s = b;
                op = opb;
            }
            if (s < 0) return 0;
            auto it = group_of.find({s, op});
            if (it != group_of.end()) return it->second;
            const int g = static_cast<int>(group_of.size()) + 1;
            group_of[{s, op}] = g;
            return g;
        };
        // list items per copy: (channel, copy) with a nonzero unrolled factor
        struct Item {
            int c, j, grp;
            double ufac;
        };
        // per copy, the far items (non-temporal loads, MRMF_TUNE_FAR_LOADS) first, then the near ones
        std::vector<std::vector<Item>> items(PU);
        std::vector<int> nfar(PU, 0);
        for (int64_t j = 0; j < PU; ++j) {
            for (int pass = 0; pass < 2; ++pass) {
                for (int c : cG) {
                    const auto& ch = P.chans[c];
                    if (far(ch.delta) != (pass == 0)) continue;
                    double u = 1.0;
                    auto mul_unrolled = [&](int s, int op) {
                        if (s >= 0 && is_unrolled(s)) u *= factor_table(p, s, op)[udigit(s, j)];
                    };
                    mul_unrolled(ch.a, ch.opa);
                    mul_unrolled(ch.b, ch.opb);
                    if (u == 0.0) continue;
                    items[j].push_back({c, static_cast<int>(j), lane_group(ch.a, ch.opa, ch.b, ch.opb), u});
                    nfar[j] += pass == 0;
                }
            }
        }
        const int NG = static_cast<int>(group_of.size()) + 2;  // + one, + sentinel
        const int ZG = NG - 1;
        int capn = 1, capf = 0, NI = 0;
        std::vector<int> ioff(PU + 1, 0);
        for (int64_t j = 0; j < PU; ++j) {
            capf = std::max<int>(capf, nfar[j]);
            capn = std::max<int>(capn, static_cast<int>(items[j].size()) - nfar[j]);
            ioff[j + 1] = ioff[j] + static_cast<int>(items[j].size());
        }
        NI = ioff[PU];
        // list of copy j in LDS: far entries at [j CAP, j CAP + n_far) followed by U sentinels (when any
        // channel is far), near entries from j CAP + NB on, followed by U sentinels
        const int NB = capf > 0 ? capf + U : 0;
        const int CAP = NB + capn + U;
        // diagonal items of the uniform kind (summed) and mixed kind (uniform part per tile)
        const int nsum = static_cast<int>(gU.size()), nmd = static_cast<int>(gM.size());

        std::ostringstream pre, o;
        const size_t one = pool_add("ONE", {1.0});
        // tables of a uniform part: up to two uniform sites (quotient magic by the site multiplier counted
        // in super-tiles, dimension and its magic, factor-table offset; an absent site has quotient magic 1,
        // hence digit 0, dimension 1 and the 1.0 entry), parameter, weight
        auto emit_tab = [&](const std::string& pfx, const std::vector<std::tuple<int, int, int, int, int, double, double>>& its,
                            const std::vector<int32_t>* soffs, const std::vector<int32_t>* grps) {
            const int n = std::max<int>(1, its.size());
            std::ostringstream mam, da, dam, ta, mbm, db, dbm, tb, pr, wr, wi, so, gr;
            for (size_t i = 0; i < its.size(); ++i) {
                std::vector<std::array<uint64_t, 3>> ss;
                for (auto sop : {std::make_pair(std::get<0>(its[i]), std::get<1>(its[i])),
                                 std::make_pair(std::get<2>(its[i]), std::get<3>(its[i]))}) {
                    if (sop.first < 0 || is_static(sop.first)) continue;
                    ss.push_back({static_cast<uint64_t>(P.M[sop.first] / STC()), static_cast<uint64_t>(P.d[sop.first]),
                                  static_cast<uint64_t>(ftab(sop.first, sop.second))});
                }
                while (ss.size() < 2) ss.push_back({0, 1, static_cast<uint64_t>(one)});
                const char* sep = i ? ", " : "";
                mam << sep << ulit(ss[0][0] == 0 ? 1 : ss[0][0] == 1 ? 0 : magic_of(ss[0][0]));
                da << sep << ss[0][1] << "u";
                dam << sep << ulit(magic_of(ss[0][1]));
                ta << sep << ss[0][2] << "u";
                mbm << sep << ulit(ss[1][0] == 0 ? 1 : ss[1][0] == 1 ? 0 : magic_of(ss[1][0]));
                db << sep << ss[1][1] << "u";
                dbm << sep << ulit(magic_of(ss[1][1]));
                tb << sep << ss[1][2] << "u";
                pr << sep << std::get<4>(its[i]);
                wr << sep << lit(std::get<5>(its[i]), f32);
                wi << sep << lit(std::get<6>(its[i]), f32);
                if (soffs) so << sep << (*soffs)[i];
                if (grps) gr << sep << (*grps)[i];
            }
            auto arr = [&](const char* ty, const char* nm, std::ostringstream& v) {
                const std::string s = v.str();
                pre << "__constant__ " << ty << " " << pfx << nm << "[" << n << "] = {" << (s.empty() ? "0" : s) << "};\n";
            };
            arr("unsigned long long", "mam", mam);
            arr("unsigned", "da", da);
            arr("unsigned long long", "dam", dam);
            arr("unsigned", "ta", ta);
            arr("unsigned long long", "mbm", mbm);
            arr("unsigned", "db", db);
            arr("unsigned long long", "dbm", dbm);
            arr("unsigned", "tb", tb);
            arr("int", "pr", pr);
            arr("R", "wr", wr);
            arr("R", "wi", wi);
            if (soffs) arr("int", "so", so);
            if (grps) arr("int", "gr", gr);
        };
        {
            std::vector<std::tuple<int, int, int, int, int, double, double>> its;
            std::vector<int32_t> soffs, grps;
            for (int64_t j = 0; j < PU; ++j)
                for (const Item& it : items[j]) {
                    const auto& ch = P.chans[it.c];
                    its.emplace_back(ch.a, ch.opa, ch.b, ch.opb, ch.param, ch.wr * it.ufac, ch.wi * it.ufac);
                    soffs.push_back(static_cast<int32_t>(copy_off(j) * sz - ch.delta * sz));
                    grps.push_back(it.grp);
                }
            emit_tab("E", its, &soffs, &grps);
            std::vector<std::tuple<int, int, int, int, int, double, double>> md, us;
            for (int g : gM) {
                const auto& dg = P.diags[g];
                md.emplace_back(dg.a, dg.opa, dg.b, dg.opb, dg.param, dg.wr, dg.wi);
            }
            for (int g : gU) {
                const auto& dg = P.diags[g];
                us.emplace_back(dg.a, dg.opa, dg.b, dg.opb, dg.param, dg.wr, dg.wi);
            }
            emit_tab("M", md, nullptr, nullptr);
            emit_tab("Q", us, nullptr, nullptr);
        }
        o << "__device__ __forceinline__ unsigned dig(unsigned t, unsigned long long mm, unsigned d, unsigned long long dm) {\n"
          << "  const unsigned q = mm ? (unsigned)__umul64hi(mm, (unsigned long long)t) : t;\n"
          << "  return q - (unsigned)__umul64hi(dm, (unsigned long long)q) * d;\n}\n";
        o << kernel_head();
        const bool dbuf = use_lds && 2 * xrows * sz <= 49152;
        if (use_lds) o << "  __shared__ C xl[" << (dbuf ? 2 : 1) * xrows << "];\n";
        o << "  __shared__ int lso[2][" << PU * CAP << "];\n"
          << "  __shared__ int lgr[2][" << PU * CAP << "];\n"
          << "  __shared__ R lcr[2][" << PU * CAP << "];\n";
        if (cplx) o << "  __shared__ R lci[2][" << PU * CAP << "];\n";
        o << "  __shared__ int lcn[2][" << PU << "];\n"
          << "  __shared__ R lfac[" << NG * block << "];\n";
        if (capf > 0) o << "  __shared__ int lcf[2][" << PU << "];\n";
        if (nmd > 0) {
            o << "  __shared__ R tr[2][" << nmd << "];\n";
            if (cplx) o << "  __shared__ R ti[2][" << nmd << "];\n";
        }
        const int swaves = std::min(nw, (nsum + 63) / 64);
        if (nsum > 0) {
            o << "  __shared__ R dsr[2][" << swaves << "];\n";
            if (cplx) o << "  __shared__ R dsi[2][" << swaves << "];\n";
        }
        o << "  __shared__ R Kl[KN_ALLOC];\n";
        o << "  const unsigned tid = threadIdx.x, wv = tid >> 6, ln = tid & 63u;\n"
          << "  const bool act = tid < " << T << "u;\n"
          << "  const unsigned r = act ? tid : 0u;\n"
          << "  const unsigned OOB = 0x80000000u;\n"
          << "  const unsigned voff = act ? r * " << sz << "u : OOB;\n";
        if (use_lds) {
            o << "  for (unsigned i = tid; i < " << halo << "u; i += " << block << "u) {\n"
              << "    const C z = {(R)0, (R)0};\n";
            for (int b = 0; b < (dbuf ? 2 : 1); ++b)
                o << "    xl[" << b * xrows << "u + i] = z; xl[" << b * xrows + halo + st << "u + i] = z;\n";
            o << "  }\n";
            for (int64_t j = 0; j < PU; ++j)
                o << "  const unsigned w" << j << " = act ? " << halo + j * T << "u + r : " << xrows - 1 << "u;\n";
        }
        o << "  for (unsigned i = tid; i < KN; i += " << block << "u) Kl[i] = K[i];\n";
        std::set<int> lane_sites, used_params;
        for (const auto& c : P.chans) {
            if (is_inner(c.a)) lane_sites.insert(c.a);
            if (c.b >= 0 && is_inner(c.b)) lane_sites.insert(c.b);
            used_params.insert(c.param);
        }
        for (const auto& g : P.diags) {
            if (is_inner(g.a)) lane_sites.insert(g.a);
            if (g.b >= 0 && is_inner(g.b)) lane_sites.insert(g.b);
            used_params.insert(g.param);
        }
        for (int s : lane_sites) o << "  const unsigned n" << s << " = (r / " << P.M[s] << "u) % " << P.d[s] << "u;\n";
        for (int q : used_params) o << "  const R th" << q << " = theta[" << q << "];\n";
        auto wexpr = [&](int param, double w) { return "th" + std::to_string(param) + " * " + lit(w, f32); };
        // per-thread group factors
        o << "  lfac[tid] = act ? (R)1 : (R)0;\n"
          << "  lfac[" << ZG * block << "u + tid] = (R)0;\n";
        for (const auto& kv : group_of)
            o << "  lfac[" << kv.second * block << "u + tid] = act ? " << lane_fac(kv.first.first, kv.first.second)
              << " : (R)0;\n";
        // static channel coefficients per copy (registers)
        std::map<std::pair<int, int64_t>, std::string> kS;
        for (int c : cS) {
            const auto& ch = P.chans[c];
            const bool unr = has_unrolled(ch.a, ch.b);
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(ch.a, ch.opa, ch.b, ch.opb, j);
                if (sp.first == 0.0) continue;
                if (!unr && j > 0 && kS.count({c, 0})) {
                    kS[{c, j}] = kS[{c, 0}];
                    continue;
                }
                const std::string nm = "k" + std::to_string(c) + "_" + std::to_string(j);
                const std::string le = sp.second.empty() ? std::string("(R)1") : sp.second;
                o << "  const R " << nm << "r = act ? " << wexpr(ch.param, ch.wr) << " * " << lit(sp.first, f32) << " * " << le
                  << " : (R)0;\n";
                if (cplx)
                    o << "  const R " << nm << "i = act ? " << wexpr(ch.param, ch.wi) << " * " << lit(sp.first, f32) << " * "
                      << le << " : (R)0;\n";
                kS[{c, j}] = nm;
            }
        }
        // static diagonal weight per copy; static factor of the mixed diagonal terms per copy
        for (int64_t j = 0; j < PU; ++j) {
            o << "  R dS" << j << "r = 0, dS" << j << "i = 0;\n";
            for (int g : gS) {
                const auto& dg = P.diags[g];
                const auto sp = static_part(dg.a, dg.opa, dg.b, dg.opb, j);
                if (sp.first == 0.0) continue;
                const std::string le = sp.second.empty() ? std::string("(R)1") : sp.second;
                o << "  { const R f = " << lit(sp.first, f32) << " * " << le << "; dS" << j << "r += " << wexpr(dg.param, dg.wr)
                  << " * f;";
                if (cplx) o << " dS" << j << "i += " << wexpr(dg.param, dg.wi) << " * f;";
                o << " }\n";
            }
        }
        std::map<std::pair<int, int64_t>, std::string> fD;
        for (int i = 0; i < nmd; ++i) {
            const auto& dg = P.diags[gM[i]];
            for (int64_t j = 0; j < PU; ++j) {
                const auto sp = static_part(dg.a, dg.opa, dg.b, dg.opb, j);
                if (sp.first == 0.0) continue;
                const std::string nm = "z" + std::to_string(i) + "_" + std::to_string(j);
                o << "  const R " << nm << " = " << lit(sp.first, f32) << " * " << (sp.second.empty() ? "(R)1" : sp.second)
                  << ";\n";
                fD[{i, j}] = nm;
            }
        }
        o << rsrc_decls(shift, nrec)
          << "  __syncthreads();\n"
          << "  const unsigned G = gridDim.x, b = blockIdx.x;\n"
          << "  unsigned par = 0u;\n";
        const bool remap = tmap("ts") != "ts";
        const std::string tv = remap ? "ts" : "t";
        if (sched == MRMF_SCHED_XCD_CHUNK) {
            o << "  const unsigned nx = (G % 8u == 0u) ? 8u : 1u, GX = G / nx, xcd = b % nx;\n"
              << "  const unsigned Cx = (" << n_st << "u + nx - 1u) / nx;\n"
              << "  const unsigned t_end = (xcd + 1u) * Cx < " << n_st << "u ? (xcd + 1u) * Cx : " << n_st << "u;\n"
              << "  const unsigned t_step = GX;\n"
              << "  unsigned " << tv << " = xcd * Cx + b / nx;\n";
        } else if (sched == MRMF_SCHED_BLOCK_RUN) {
            o << "  const unsigned v = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;\n"
              << "  const unsigned t_end = (unsigned)(((unsigned long long)(v + 1u) * " << n_st << "ull) / G), t_step = 1u;\n"
              << "  unsigned " << tv << " = (unsigned)(((unsigned long long)v * " << n_st << "ull) / G);\n";
        } else {
            o << "  const unsigned t_end = " << n_st << "u, t_step = G;\n"
              << "  unsigned " << tv << " = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;\n";
        }
        auto soff = [&](int64_t j, int64_t delta, const std::string& base) { return soff_expr(base, j, delta); };
        // self rows of the first super-tile
        for (int64_t j = 0; j < PU; ++j)
            o << "  C xn" << j << " = {(R)0, (R)0};\n";
        o << "  if (" << tv << " < t_end) {\n    " << base_decl("Fn", tmap(tv), shift) << "\n";
        for (int64_t j = 0; j < PU; ++j) o << "    xn" << j << " = LD(xs, voff, " << soff(j, 0, "Fn") << ");\n";
        o << "  }\n";
        o << "  for (; " << tv << " < t_end; " << tv << " += t_step) {\n";
        if (remap) o << "    const unsigned t = " << tmap("ts") << ";\n";
        o << "    " << base_decl("F0", "t", shift) << "\n";
        for (int64_t j = 0; j < PU; ++j) o << "    const C x" << j << " = xn" << j << ";\n";
        if (use_lds) {
            o << "    C* lb = xl" << (dbuf ? " + par * " + std::to_string(xrows) + "u" : std::string("")) << ";\n";
            for (int64_t j = 0; j < PU; ++j) o << "    lb[w" << j << "] = x" << j << ";\n";
        }
        // list construction: wave w builds the lists of copies j = w, w + nw, ...
        if (NI > 0) {
            const std::string sentinel = std::string("lso[par][q] = 0; lgr[par][q] = ") + std::to_string(ZG) +
                                         "; lcr[par][q] = (R)0;" + (cplx ? " lci[par][q] = (R)0;" : "");
            o << "    for (unsigned j = wv; j < " << PU << "u; j += " << nw << "u) {\n"
              << "      unsigned base = 0u;\n"
              << (capf > 0 ? "      unsigned basef = 0u;\n      const unsigned nfi = Enf[j];\n" : "")
              << "      const unsigned i0 = Eoff[j], ni = Eoff[j + 1u] - i0;\n"
              << "      for (unsigned h = 0u; h < ni; h += 64u) {\n"
              << "        const unsigned i = h + ln;\n"
              << "        const bool has = i < ni;\n"
              << "        const unsigned e = i0 + (has ? i : 0u);\n"
              << "        const unsigned na = dig(t, Emam[e], Eda[e], Edam[e]), nb = dig(t, Embm[e], Edb[e], Edbm[e]);\n"
              << "        const R f = Kl[Eta[e] + na] * Kl[Etb[e] + nb];\n"
              << "        const bool adm = has && f != (R)0;\n";
            if (capf > 0)
                o << "        const bool isf = i < nfi;\n"
                  << "        const unsigned long long m = __ballot(adm && !isf), mf = __ballot(adm && isf);\n"
                  << "        if (adm) {\n"
                  << "          const unsigned long long lt = (1ull << ln) - 1ull;\n"
                  << "          const unsigned q = j * " << CAP << "u + (isf ? basef + (unsigned)__popcll(mf & lt) : "
                  << NB << "u + base + (unsigned)__popcll(m & lt));\n";
            else
                o << "        const unsigned long long m = __ballot(adm);\n"
                  << "        if (adm) {\n"
                  << "          const unsigned pos = base + (unsigned)__popcll(m & ((1ull << ln) - 1ull));\n"
                  << "          const unsigned q = j * " << CAP << "u + pos;\n";
            o << "          const R th = theta[Epr[e]] * f;\n"
              << "          lso[par][q] = Eso[e]; lgr[par][q] = Egr[e]; lcr[par][q] = th * Ewr[e];\n"
              << (cplx ? "          lci[par][q] = th * Ewi[e];\n" : "")
              << "        }\n"
              << "        base += (unsigned)__popcll(m);\n"
              << (capf > 0 ? "        basef += (unsigned)__popcll(mf);\n" : "")
              << "      }\n"
              << "      if (ln < " << U << "u) {\n"
              << "        { const unsigned q = j * " << CAP << "u + " << NB << "u + base + ln; " << sentinel << " }\n"
              << (capf > 0 ? "        { const unsigned q = j * " + std::to_string(CAP) + "u + basef + ln; " + sentinel + " }\n"
                           : std::string(""))
              << "      }\n"
              << "      if (ln == 0u) { lcn[par][j] = base;" << (capf > 0 ? " lcf[par][j] = basef;" : "") << " }\n"
              << "    }\n";
            std::ostringstream eo, fo;
            for (int64_t j = 0; j <= PU; ++j) eo << (j ? ", " : "") << ioff[j] << "u";
            pre << "__constant__ unsigned Eoff[" << PU + 1 << "] = {" << eo.str() << "};\n";
            if (capf > 0) {
                for (int64_t j = 0; j < PU; ++j) fo << (j ? ", " : "") << nfar[j] << "u";
                pre << "__constant__ unsigned Enf[" << PU << "] = {" << fo.str() << "};\n";
            }
        }
        // mixed diagonal uniform parts and the uniform diagonal sum (first waves)
        if (nmd > 0) {
            o << "    for (unsigned i = tid; i < " << nmd << "u; i += " << block << "u) {\n"
              << "      const unsigned na = dig(t, Mmam[i], Mda[i], Mdam[i]), nb = dig(t, Mmbm[i], Mdb[i], Mdbm[i]);\n"
              << "      const R f = theta[Mpr[i]] * Kl[Mta[i] + na] * Kl[Mtb[i] + nb];\n"
              << "      tr[par][i] = f * Mwr[i];\n"
              << (cplx ? "      ti[par][i] = f * Mwi[i];\n" : "")
              << "    }\n";
        }
        if (nsum > 0) {
            o << "    if (wv < " << swaves << "u) {\n"
              << "      R vr = (R)0, vi = (R)0;\n"
              << "      for (unsigned i = tid; i < " << nsum << "u; i += " << swaves * 64 << "u) {\n"
              << "        const unsigned ma = dig(t, Qmam[i], Qda[i], Qdam[i]), mb = dig(t, Qmbm[i], Qdb[i], Qdbm[i]);\n"
              << "        const R g = theta[Qpr[i]] * Kl[Qta[i] + ma] * Kl[Qtb[i] + mb];\n"
              << "        vr += g * Qwr[i]; vi += g * Qwi[i];\n"
              << "      }\n"
              << "      for (int k = 32; k > 0; k >>= 1) { vr += __shfl_down(vr, k, 64);"
              << (cplx ? " vi += __shfl_down(vi, k, 64);" : "") << " }\n"
              << "      if (ln == 0u) { dsr[par][wv] = vr;" << (cplx ? " dsi[par][wv] = vi;" : "") << " }\n"
              << "    }\n";
        }
        o << "    __syncthreads();\n";
        // prefetch the self rows of the next super-tile
        o << "    if (" << tv << " + t_step < t_end) {\n      " << base_decl("Fn", tmap(tv + " + t_step"), shift) << "\n";
        for (int64_t j = 0; j < PU; ++j) o << "      xn" << j << " = LD(xs, voff, " << soff(j, 0, "Fn") << ");\n";
        o << "    }\n";
        o << "    R dUr = (R)0, dUi = (R)0;\n";
        for (int w = 0; w < (nsum > 0 ? swaves : 0); ++w)
            o << "    dUr += dsr[par][" << w << "];" << (cplx ? " dUi += dsi[par][" + std::to_string(w) + "];" : "") << "\n";
        auto acc = [&](int64_t j, const std::string& kr, const std::string& ki, const std::string& s) {
            o << "a" << j << "r += " << kr << " * " << s << ".x; a" << j << "i += " << kr << " * " << s << ".y;";
            if (!ki.empty()) o << " a" << j << "r -= " << ki << " * " << s << ".y; a" << j << "i += " << ki << " * " << s << ".x;";
        };
        for (int64_t j = 0; j < PU; ++j) {
            o << "    {\n      R a" << j << "r, a" << j << "i;\n      {\n        R dr = dS" << j << "r + dUr, di = dS" << j
              << "i + dUi;\n";
            for (int i = 0; i < nmd; ++i) {
                auto it = fD.find({i, j});
                if (it == fD.end()) continue;
                o << "        dr += tr[par][" << i << "] * " << it->second << ";";
                if (cplx) o << " di += ti[par][" << i << "] * " << it->second << ";";
                o << "\n";
            }
            o << "        a" << j << "r = dr * x" << j << ".x - di * x" << j << ".y; a" << j << "i = dr * x" << j << ".y + di * x" << j
              << ".x;\n      }\n";
            if (use_lds) {
                for (int c : cS) {
                    auto it = kS.find({c, j});
                    if (it == kS.end()) continue;
                    const int64_t off = halo + j * T - lds_delta(c);
                    o << "      { const C s = lb[r + " << off << "u]; ";
                    acc(j, it->second + "r", cplx ? it->second + "i" : "", "s");
                    o << " }\n";
                }
            }
            // walk one sublist of copy j's list in chunks of U gathers (LD, or LDN for the far entries)
            auto walk = [&](const std::string& count, int64_t start, const char* ld) {
                o << "      { const unsigned n = (unsigned)__builtin_amdgcn_readfirstlane(" << count << ");\n"
                  << "      for (unsigned k = " << start << "u; k < " << start << "u + n; k += " << U << "u) {\n";
                for (int u = 0; u < U; ++u)
                    o << "        const int so" << u << " = __builtin_amdgcn_readfirstlane(lso[par][k + " << u << "u]);"
                      << " const int g" << u << " = __builtin_amdgcn_readfirstlane(lgr[par][k + " << u << "u]);"
                      << " const R f" << u << " = lfac[(unsigned)g" << u << " * " << block << "u + tid];"
                      << " const C s" << u << " = " << ld << "(xs, f" << u << " != (R)0 ? voff : OOB, F0 + "
                      << (wide ? "(unsigned long long)(long long)so" : "(unsigned)so") << u << ");\n";
                for (int u = 0; u < U; ++u) {
                    o << "        { const R cr = lcr[par][k + " << u << "u] * f" << u << ";";
                    if (cplx) o << " const R ci = lci[par][k + " << u << "u] * f" << u << ";";
                    o << " ";
                    acc(j, "cr", cplx ? "ci" : "", "s" + std::to_string(u));
                    o << " }\n";
                }
                o << "      } }\n";
            };
            if (NI > 0) {
                if (capf > 0) walk("lcf[par][" + std::to_string(j) + "]", j * CAP, "LDN");
                walk("lcn[par][" + std::to_string(j) + "]", j * CAP + NB, "LD");
            }
            o << store_out("      ", j, soff(j, 0, "F0"), false) << "    }\n";
        }
        if (!dbuf) o << "    __syncthreads();\n";
        o << "    par ^= 1u;\n  }\n}\n";

        std::ostringstream full;
        full << "// generated (list form): " << P.N << " sites, " << nch << " channels (" << cS.size() << " static, " << cG.size()
             << " listed), " << ndg << " diagonal terms; " << T << " rows per block (sites " << tl.k_in << ".." << P.N - 1
             << "), " << PU << " unrolled copies (sites " << tl.k_u << ".." << tl.k_in - 1 << "), " << n_st
             << " super-tiles\n";
        full << prelude();
        full << "#define KN " << pool.size() << "u\n#define KN_ALLOC " << std::max<size_t>(pool.size(), 1) << "\n";
        full << "__constant__ R K[" << std::max<size_t>(pool.size(), 1) << "] = {";
        if (pool.empty()) full << "0";
        for (size_t i = 0; i < pool.size(); ++i) full << (i ? ", " : "") << lit(pool[i], f32);
        full << "};\n" << pre.str() << o.str();
        return full.str();
    }
};

// Tile choice.  Inner block: the low sites with T_in <= 1024 rows, preferring blocks of at least 256
// rows that fill whole wavefronts.  Unrolled copies: the next sites up while P_U <= 4 and at least 2048
// super-tiles remain to fill the GPU.
bool choose_tiling(const mrmf_plan_t* p, int inner_pref, int unroll_pref, int unroll_top, Tile* tl) {
    const int N = p->N;
    int k_in = N;
    int64_t T = 1;
    if (inner_pref > 0) {
        if (inner_pref > N) return false;
        for (int i = N - inner_pref; i < N; ++i) T *= p->d[i];
        if (T > 1024) return false;
        k_in = N - inner_pref;
    } else {
        double best = -1.0;
        int64_t t = 1;
        for (int k = N - 1; k >= 0; --k) {
            t *= p->d[k];
            if (t > 1024) break;
            const double eff = double(t) / double(round_up(t, 64));
            const double score = eff * std::min(1.0, double(t) / 256.0);
            if (score > best + 1e-12) {
                best = score;
                k_in = k;
                T = t;
            }
        }
        if (best < 0) return false;
    }
    int k_u = k_in;
    int64_t PU = 1;
    if (unroll_pref >= 0) {
        for (int i = 0; i < unroll_pref && k_u > 0; ++i) PU *= p->d[--k_u];
        if (PU > 16) return false;
    } else {
        while (k_u > 0 && PU * p->d[k_u - 1] <= 4 && p->D / (T * PU * p->d[k_u - 1]) >= 2048) PU *= p->d[--k_u];
    }
    tl->k_in = k_in;
    tl->k_u = k_u;
    tl->T_in = T;
    tl->P_C = PU;
    tl->n_top = 0;
    if (unroll_top > 0 && k_u > unroll_top) {  // sites 0..unroll_top-1 unrolled too; a uniform site remains
        for (int s = 0; s < unroll_top; ++s) PU *= p->d[s];
        if (PU > 16) return false;
        tl->n_top = unroll_top;
    }
    tl->P_U = PU;
    return true;
}

}  // namespace

// Adjoint kernel generated for one plan (c128, Hermitian groups).  For an upstream gradient g the adjoint
// needs grad_x = H g and grad_theta_p = Re <g | h_p x> = Re <h_p g | x> (h_p Hermitian), and both come from
// the terms of the gather form (Sec. II) applied to g:
//     t = w f(F) g[F - Delta],   grad_x[F] += theta_p t,   grad_theta_p += Re conj(t) x_F.
// The plan is compiled in: digits from the row index by shifts or by multiplication with compile-time
// reciprocals (Eq. decode), each one-site factor table <n|O|n - q> as a select over literals (d <= 3) or an
// LDS table, one register accumulator per parameter.  A zero factor (inadmissible source) masks its gather
// to the out-of-range offset, which reads zero.  The channels are taken in groups whose gathers are all
// issued before any of them is used (a scheduling barrier keeps them together), so a row waits for memory
// once per group.  Each thread sums its rows; at the end every parameter is summed over the wave by a fixed
// pattern of DPP moves and over the block's four waves in a fixed order into partial[block * n_params + p],
// so the result does not depend on scheduling.  "" when the plan has no parameters, more than
// kGradMaxParams, or a vector of 2^31 bytes or more.
std::string grad_source(const mrmf_plan_t* p) {
    const int np = p->n_params, N = p->N;
    if (np < 1 || np > kGradMaxParams || p->D * 16 >= (int64_t(1) << 31)) return "";
    std::vector<double> lds;                       // tables of sites with d > 3
    std::map<std::pair<int, int>, size_t> lds_at;  // (site, op) -> offset in lds
    // one-site factor <n|O|n - q> at the row's digit of `site`, as an expression
    auto factor = [&](int site, int op) -> std::string {
        const int d = p->d[site];
        const std::string n = "n" + std::to_string(site);
        std::ostringstream e;
        if (d == 1) {
            e << lit(local_factor_host(p, site, op, 0), false);
        } else if (d <= 3) {
            e << "(" << n << " == 0u ? " << lit(local_factor_host(p, site, op, 0), false) << " : ";
            if (d == 2) {
                e << lit(local_factor_host(p, site, op, 1), false) << ")";
            } else {
                e << "(" << n << " == 1u ? " << lit(local_factor_host(p, site, op, 1), false) << " : "
                  << lit(local_factor_host(p, site, op, 2), false) << "))";
            }
        } else {
            auto it = lds_at.find({site, op});
            if (it == lds_at.end()) {
                it = lds_at.emplace(std::make_pair(site, op), lds.size()).first;
                for (int v = 0; v < d; ++v) lds.push_back(local_factor_host(p, site, op, v));
            }
            e << "Kl[" << it->second << "u + " << n << "]";
        }
        return e.str();
    };
    struct T {
        int a, opa, b, opb, param;
        double wr, wi;
        int64_t delta;
        bool diag;
    };
    std::vector<T> terms;
    for (const auto& g : p->diags) terms.push_back({g.a, g.opa, g.b, g.opb, g.param, g.wr, g.wi, 0, true});
    for (const auto& c : p->chans) terms.push_back({c.a, c.opa, c.b, c.opb, c.param, c.wr, c.wi, c.delta, false});
    std::set<int> used;
    for (const T& t : terms) {
        used.insert(t.a);
        if (t.b >= 0) used.insert(t.b);
    }
    std::set<int> params_used;
    for (const T& t : terms) params_used.insert(t.param);
    // accumulation of term k with source value sk (complex) and factor fk
    auto accumulate = [&](std::ostringstream& o, const T& t, const std::string& f, const std::string& s) {
        o << "      { const double c = " << f << " * " << lit(t.wr, false) << ";";
        if (t.wi == 0.0) {
            o << " const double e = c * th" << t.param << ";"
              << " hr = fma(e, " << s << ".x, hr); hi = fma(e, " << s << ".y, hi);"
              << " a" << t.param << " = fma(c, " << s << ".x * xf.x + " << s << ".y * xf.y, a" << t.param << "); }\n";
        } else {
            o << " const double ci = " << f << " * " << lit(t.wi, false) << ";"
              << " const double tr = c * " << s << ".x - ci * " << s << ".y, ti = c * " << s << ".y + ci * " << s << ".x;"
              << " hr = fma(th" << t.param << ", tr, hr); hi = fma(th" << t.param << ", ti, hi);"
              << " a" << t.param << " = fma(tr, xf.x, fma(ti, xf.y, a" << t.param << ")); }\n";
        }
    };
    auto fexpr = [&](const T& t) {
        std::string f = factor(t.a, t.opa);
        if (t.b >= 0) f = "(" + f + " * " + factor(t.b, t.opb) + ")";
        return f;
    };
    std::ostringstream body;
    // diagonal terms: the source is g_F itself
    for (const T& t : terms)
        if (t.diag) accumulate(body, t, fexpr(t), "gf");
    // channels in groups of at most kGroup gathers
    std::vector<const T*> ch;
    for (const T& t : terms)
        if (!t.diag) ch.push_back(&t);
    constexpr int kGroup = 24;
    const int ngr = static_cast<int>((ch.size() + kGroup - 1) / kGroup);
    const int gsz = ngr > 0 ? static_cast<int>((ch.size() + ngr - 1) / ngr) : 0;
    for (size_t g0 = 0; g0 < ch.size(); g0 += gsz) {
        const size_t g1 = std::min(ch.size(), g0 + gsz);
        body << "    {\n";
        for (size_t k = g0; k < g1; ++k)
            body << "      const double f" << k - g0 << " = " << fexpr(*ch[k]) << ";\n";
        for (size_t k = g0; k < g1; ++k)
            body << "      const C s" << k - g0 << " = LD(gs, f" << k - g0 << " != 0.0 ? vf - " << ch[k]->delta * 16
                 << "u : OOB);\n";
        body << "      __builtin_amdgcn_sched_barrier(0);\n";
        for (size_t k = g0; k < g1; ++k)
            accumulate(body, *ch[k], "f" + std::to_string(k - g0), "s" + std::to_string(k - g0));
        body << "    }\n";
    }
    std::ostringstream o;
    o << "// generated adjoint kernel: " << N << " sites, " << p->diags.size() << " diagonal terms, " << p->chans.size()
      << " channels, " << np << " parameters\n";
    o << "typedef double C __attribute__((ext_vector_type(2)));\n"
      << "typedef unsigned U2 __attribute__((ext_vector_type(2)));\n"
      << "typedef unsigned U4 __attribute__((ext_vector_type(4)));\n"
      << "#define LD(rs, vo) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128((rs), (int)(vo), 0, 0))\n"
      << "#define OOB 0x80000000u\n";
    if (!lds.empty()) {
        o << "__constant__ double K[" << lds.size() << "] = {";
        for (size_t i = 0; i < lds.size(); ++i) o << (i ? ", " : "") << lit(lds[i], false);
        o << "};\n";
    }
    o << "// v moved across lanes by one DPP pattern (rows outside row_mask take 0), one 32-bit half at a time\n"
      << "template <int CTRL, int ROW_MASK>\n__device__ __forceinline__ double dpp_move(double v) {\n"
      << "  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);\n"
      << "  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROW_MASK, 0xf, false);\n"
      << "  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROW_MASK, 0xf, false);\n"
      << "  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);\n}\n"
      << "// sum over the 64 lanes (pairs, quads, half-row and row mirrors, row broadcasts 15 and 31): lane 63\n"
      << "__device__ __forceinline__ double wave_sum(double v) {\n"
      << "  v += dpp_move<0xB1, 0xf>(v);\n  v += dpp_move<0x4E, 0xf>(v);\n  v += dpp_move<0x141, 0xf>(v);\n"
      << "  v += dpp_move<0x140, 0xf>(v);\n  v += dpp_move<0x142, 0xa>(v);\n  v += dpp_move<0x143, 0xc>(v);\n"
      << "  return v;\n}\n";
    o << "extern \"C\" __global__ __launch_bounds__(256) void mrmf_grad(const double* __restrict__ theta,\n"
      << "    const C* __restrict__ x, const C* __restrict__ g, C* __restrict__ gx, double* __restrict__ partial) {\n"
      << "  __shared__ double red[" << np << "][4];\n";
    if (!lds.empty())
        o << "  __shared__ double Kl[" << lds.size() << "];\n"
          << "  for (unsigned i = threadIdx.x; i < " << lds.size() << "u; i += 256u) Kl[i] = K[i];\n"
          << "  __syncthreads();\n";
    o << "  const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, " << p->D * 16
      << ", 0x00020000);\n"
      << "  const __amdgpu_buffer_rsrc_t gs = __builtin_amdgcn_make_buffer_rsrc((void*)g, (short)0, " << p->D * 16
      << ", 0x00020000);\n"
      << "  const __amdgpu_buffer_rsrc_t os = __builtin_amdgcn_make_buffer_rsrc((void*)gx, (short)0, " << p->D * 16
      << ", 0x00020000);\n"
      << "  const unsigned tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;\n";
    for (int q : params_used) o << "  const double th" << q << " = theta[" << q << "];\n";
    for (int q = 0; q < np; ++q) o << "  double a" << q << " = 0.0;\n";
    o << "  for (unsigned F = blockIdx.x * 256u + tid; F < " << p->D << "u; F += gridDim.x * 256u) {\n"
      << "    const unsigned vf = F * 16u;\n"
      << "    unsigned f = F;\n";
    for (int i = N - 1; i >= 0; --i) {  // Eq. decode, least significant site first
        const uint64_t d = static_cast<uint64_t>(p->d[i]);
        const std::string I = std::to_string(i);
        const bool use = used.count(i) != 0;
        if (d == 1) {
            if (use) o << "    const unsigned n" << I << " = 0u;\n";
        } else if (i == 0) {
            if (use) o << "    const unsigned n0 = f;\n";
        } else if ((d & (d - 1)) == 0) {
            if (use) o << "    const unsigned n" << I << " = f & " << d - 1 << "u;";
            else o << "   ";
            o << " f >>= " << __builtin_ctzll(d) << "u;\n";
        } else if (use) {
            o << "    const unsigned q" << I << " = (unsigned)__umul64hi(" << ulit(magic_of(d)) << ", (unsigned long long)f);\n"
              << "    const unsigned n" << I << " = f - q" << I << " * " << d << "u; f = q" << I << ";\n";
        } else {
            o << "    f = (unsigned)__umul64hi(" << ulit(magic_of(d)) << ", (unsigned long long)f);\n";
        }
    }
    o << "    const C gf = LD(gs, vf), xf = LD(xs, vf);\n"
      << "    double hr = 0.0, hi = 0.0;\n"
      << body.str()
      << "    { C out; out.x = hr; out.y = hi;\n"
      << "      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, out), os, (int)vf, 0, 2); }\n"
      << "  }\n";
    for (int q = 0; q < np; ++q)
        o << "  { const double v = wave_sum(a" << q << "); if (lane == 63u) red[" << q << "][wave] = v; }\n";
    o << "  __syncthreads();\n"
      << "  const __amdgpu_buffer_rsrc_t ps = __builtin_amdgcn_make_buffer_rsrc((void*)partial, (short)0, gridDim.x * "
      << np * 8 << "u, 0x00020000);\n"
      << "  if (tid < " << np << "u) {\n"
      << "    const double v = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];\n"
      << "    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), ps, (int)((blockIdx.x * " << np
      << "u + tid) * 8u), 0, 0);\n"
      << "  }\n"
      << "}\n";
    return o.str();
}

// Sector kernel generated for one digit-sum sector (Sec. VI, case 2; App. D) and element type.  One
// thread per packed row r.  The row's digits come from the packed-digit table of the workspace (one word per
// state, filled from the combinatorial rank tables when the workspace is uploaded) instead of unranking r,
// and the remaining sums q_k = Q - n_0 - .. - n_{k-1} from the digits.  Then the diagonal terms and every
// sum-preserving channel on sites i < j, whose source rank is r plus the change of the rank-table terms of
// sites i..j (the remaining sums q_k, i < k <= j, move by the channel's shift at site i).
//
// Coefficients come from tables in LDS that every block fills once from theta: per channel the value
// theta_p w <n_a|O_a|n_a - q_a> <n_b|O_b|n_b - q_b> for every pair of target digits, per pair of sites the
// sum of the diagonal terms on them (one-site terms folded into a pair that contains their site), so a row
// reads one table entry per channel and per site pair instead of evaluating factor products.
//
// Rank changes come from LDS tables too.  A channel's span i..j is cut into segments of two adjacent sites
// (one for the last site of an odd span) from i on; a segment's table, indexed by (q, digits) of its first
// site and the digit of its second, holds its sites' share of the change times SZ (a byte offset).
// Channels of the same span share the segment indices and have their tables interleaved, so one LDS read
// serves two of them.  When the span is one segment (adjacent sites) the entry is the whole offset, or 2^31
// where a source digit leaves its range: the buffer load then lands past the end of x (whose byte size is
// below 2^31) and returns zero, so such a channel needs no digit checks.  Longer spans add their segments in
// 32-bit unsigned arithmetic (exact modulo 2^32; the true offset lies within +-2^31) and are masked to that
// out-of-range offset by integer checks of their source digits.  Gathers are issued in groups behind a
// scheduling barrier.
std::string sector_source(const mrmf_sector_t* S, int dtype, bool epi) {
    const bool f32 = dtype == MRMF_DTYPE_C;
    const int N = S->N, Q = S->Q, SZ = f32 ? 8 : 16;
    if (N < 1 || N > 64 || S->Dr < 1 || S->Dr * SZ >= (int64_t(1) << 31) || S->lab_bytes == 0) return "";
    if (epi && f32) return "";  // the Chebyshev step is a c128 form
    const int nch = static_cast<int>(S->chans.size());
    // factor tables <n|O|n - q> at the target digit, in the order they were built (diagonal terms, then
    // channels; site a then site b)
    size_t at = 0;
    auto take = [&](int site) {
        const int d = S->d[site];
        std::vector<double> t(S->tfac.begin() + static_cast<std::ptrdiff_t>(at),
                              S->tfac.begin() + static_cast<std::ptrdiff_t>(at + d));
        at += d;
        return t;
    };
    struct Contrib {
        int param;
        double vr, vi;
    };
    std::vector<std::vector<Contrib>> ent;  // coefficient-table entries, each a sum over parameters
    bool cplx = false;
    auto add = [&](size_t e, int param, double vr, double vi) {
        if (vr == 0.0 && vi == 0.0) return;
        cplx |= vi != 0.0;
        for (auto& c : ent[e])
            if (c.param == param) {
                c.vr += vr;
                c.vi += vi;
                return;
            }
        ent[e].push_back({param, vr, vi});
    };
    // diagonal tables, keyed by (lo, hi) site pairs (hi = -1: one site); one-site terms join a pair that
    // contains their site when there is one
    const int ndg = static_cast<int>(S->diags.size());
    std::vector<std::vector<double>> dfa(ndg), dfb(ndg);
    for (int g = 0; g < ndg; ++g) {
        dfa[g] = take(S->diags[g].a);
        if (S->diags[g].b >= 0) dfb[g] = take(S->diags[g].b);
    }
    std::map<std::pair<int, int>, size_t> doff;  // key -> offset of its table in ent
    std::vector<std::pair<int, int>> dkeys;
    auto key_table = [&](std::pair<int, int> key) {
        auto it = doff.find(key);
        if (it != doff.end()) return it->second;
        const size_t off = ent.size();
        const int n = S->d[key.first] * (key.second >= 0 ? S->d[key.second] : 1);
        ent.resize(off + n);
        doff[key] = off;
        dkeys.push_back(key);
        return off;
    };
    for (int g = 0; g < ndg; ++g) {
        const DevDiag& t = S->diags[g];
        if (t.b >= 0) key_table({std::min(t.a, t.b), std::max(t.a, t.b)});
    }
    for (int g = 0; g < ndg; ++g) {
        const DevDiag& t = S->diags[g];
        std::pair<int, int> key{t.a, -1};
        if (t.b >= 0) {
            key = {std::min(t.a, t.b), std::max(t.a, t.b)};
        } else {
            for (const auto& k : dkeys)
                if (k.second >= 0 && (k.first == t.a || k.second == t.a)) {
                    key = k;
                    break;
                }
        }
        const size_t off = key_table(key);
        const int dlo = S->d[key.first], dhi = key.second >= 0 ? S->d[key.second] : 1;
        for (int nl = 0; nl < dlo; ++nl)
            for (int nh = 0; nh < dhi; ++nh) {
                // digits of the term's sites within the key
                const int na = t.a == key.first ? nl : nh;
                double f = dfa[g][na];
                if (t.b >= 0) f *= dfb[g][t.b == key.first ? nl : nh];
                add(off + size_t(nl) * dhi + nh, t.param, t.wr * f, t.wi * f);
            }
    }
    // channel tables: entry (n_a, n_b) at co[c] + n_a d_b + n_b
    std::vector<size_t> co(nch);
    for (int c = 0; c < nch; ++c) {
        const DevChan& ch = S->chans[c];
        const std::vector<double> fa = take(ch.a), fb = take(ch.b);
        const int da = S->d[ch.a], db = S->d[ch.b];
        co[c] = ent.size();
        ent.resize(ent.size() + size_t(da) * db);
        for (int na = 0; na < da; ++na)
            for (int nb = 0; nb < db; ++nb) add(co[c] + size_t(na) * db + nb, ch.param, ch.wr * fa[na] * fb[nb],
                                                ch.wi * fa[na] * fb[nb]);
    }
    const size_t NE = std::max<size_t>(1, ent.size());
    if (NE * (f32 ? 4 : 8) * (cplx ? 2 : 1) > 32 * 1024) return "";
    std::vector<int32_t> cb{0}, cp;
    std::vector<double> cvr, cvi;
    for (const auto& e : ent) {
        for (const auto& c : e) {
            cp.push_back(c.param);
            cvr.push_back(c.vr);
            cvi.push_back(c.vi);
        }
        cb.push_back(static_cast<int32_t>(cp.size()));
    }

    // rank-change segment tables
    struct Span {
        int i, j, si, sj;  // sites i < j; source digits n_i - si, n_j - sj
    };
    std::vector<Span> sp(nch);
    for (int c = 0; c < nch; ++c) {
        const DevChan& ch = S->chans[c];
        const bool a_first = ch.a < ch.b;
        sp[c] = {a_first ? ch.a : ch.b, a_first ? ch.b : ch.a, a_first ? ch.qa : ch.qb, a_first ? ch.qb : ch.qa};
    }
    // R_k(q, v), zero outside q in 0 .. Q, v in 0 .. d_k
    auto R = [&](int k, int q, int v) -> int64_t {
        if (q < 0 || q > Q || v < 0 || v > S->d[k]) return 0;
        return S->rt[S->rto[k] + int64_t(q) * (S->d[k] + 1) + v];
    };
    // site k's share of channel c's rank change at target (q_k, n_k)
    auto share = [&](const Span& z, int k, int q, int n) -> int64_t {
        if (k == z.i) return R(k, q, n - z.si) - R(k, q, n);
        if (k < z.j) return R(k, q + z.si, n) - R(k, q, n);
        return R(k, q + z.si, n - z.sj) - R(k, q, n);
    };
    // groups of at most two channels with the same span, in channel order
    std::vector<std::vector<int>> groups;
    {
        std::map<std::pair<int, int>, int> open;  // span -> group with one member
        for (int c = 0; c < nch; ++c) {
            const std::pair<int, int> key{sp[c].i, sp[c].j};
            auto it = open.find(key);
            if (it != open.end()) {
                groups[it->second].push_back(c);
                open.erase(it);
            } else {
                open[key] = static_cast<int>(groups.size());
                groups.push_back({c});
            }
        }
    }
    std::vector<uint32_t> seg;                     // all segment tables
    std::vector<std::vector<size_t>> gso(groups.size());  // per group, offset of each segment's table
    for (size_t g = 0; g < groups.size(); ++g) {
        const Span& z0 = sp[groups[g][0]];
        const int gp = static_cast<int>(groups[g].size());
        const bool single = z0.j == z0.i + 1;
        for (int s = z0.i; s <= z0.j; s += 2) {
            const bool pair = s + 1 <= z0.j;
            const int ds = S->d[s], dt = pair ? S->d[s + 1] : 1;
            if (seg.size() % 2) seg.push_back(0);  // 8-byte aligned tables for two-channel reads
            gso[g].push_back(seg.size());
            for (int q = 0; q <= Q; ++q)
                for (int n = 0; n < ds; ++n)
                    for (int m = 0; m < dt; ++m)
                        for (int u = 0; u < gp; ++u) {
                            const Span& z = sp[groups[g][u]];
                            int64_t e = share(z, s, q, n);
                            if (pair) e += share(z, s + 1, q - n, m);
                            uint32_t v = static_cast<uint32_t>(e * SZ);
                            if (single) {
                                const bool ok = n - z.si >= 0 && n - z.si < ds && m - z.sj >= 0 && m - z.sj < dt && n <= q;
                                v = ok ? v : 0x80000000u;
                            }
                            seg.push_back(v);
                        }
        }
    }
    if (seg.size() * 4 > 40 * 1024) return "";

    const int kGroup = S->group > 0 ? S->group : 16;
    std::vector<int> pending;
    std::ostringstream body;
    auto flush = [&](bool last) {
        if (pending.empty()) return;
        body << "    __builtin_amdgcn_sched_barrier(0);\n";
        for (int c : pending) {
            const std::string u = std::to_string(c);
            body << "    { const R cr = Tr[" << co[c] << "u + x" << u << "]; ar = fma(cr, s" << u << ".x, ar); ai = fma(cr, s" << u
                 << ".y, ai);";
            if (cplx)
                body << " const R ci = Ti[" << co[c] << "u + x" << u << "]; ar = fma(-ci, s" << u << ".y, ar); ai = fma(ci, s" << u
                     << ".x, ai);";
            body << " }\n";
        }
        if (!last) body << "    MRMF_GROUP_FENCE(ar, ai);\n";
        pending.clear();
    };
    const bool w64 = S->lab_bytes == 8;
    body << "    R dr = (R)0, di = (R)0, ar = (R)0, ai = (R)0;\n"
         << "    const unsigned rb = r * " << SZ << "u;\n"
         << "    const C xf = LD(xs, rb);\n";
    if (w64)
        body << "    const unsigned long long lw = __builtin_bit_cast(unsigned long long, "
                "__builtin_amdgcn_raw_buffer_load_b64(ls, (int)(r * 8u), 0, 0));\n";
    else
        body << "    const unsigned lw = __builtin_amdgcn_raw_buffer_load_b32(ls, (int)(r * 4u), 0, 0);\n";
    if (nch > 0) {
        body << "    unsigned ";
        for (int c = 0; c < nch; ++c) body << (c ? ", " : "") << "e" << c << " = 0u";
        body << ";\n";
    }
    // bit offset of site k's digit in the packed word (site N - 1 lowest)
    std::vector<int> off(N, 0);
    for (int k = N - 2; k >= 0; --k) off[k] = off[k + 1] + S->lab_w[k + 1];
    for (int k = 0; k < N; ++k) {
        const std::string K = std::to_string(k);
        // digit and remaining sum of site k (q_k in 0 .. Q: 24-bit multiplies for the table indices)
        if (S->lab_w[k] > 0)
            body << "    const int n" << K << " = (int)((lw >> " << off[k] << ") & " << ((1u << S->lab_w[k]) - 1) << "u);\n";
        else
            body << "    const int n" << K << " = 0;\n";
        if (k == 0)
            body << "    const int q0 = " << Q << ";\n";
        else
            body << "    const int q" << K << " = q" << k - 1 << " - n" << k - 1 << ";\n";
        body << "    __builtin_assume((unsigned)q" << K << " <= " << Q << "u);\n";
        for (const auto& key : dkeys) {
            if (std::max(key.first, key.second) != k) continue;
            const size_t o = doff[key];
            body << "    { const unsigned e = " << o << "u + ";
            if (key.second >= 0) body << "(unsigned)n" << key.first << " * " << S->d[key.second] << "u + (unsigned)n" << key.second;
            else body << "(unsigned)n" << key.first;
            body << "; dr += Tr[e];" << (cplx ? " di += Ti[e];" : "") << " }\n";
        }
        // segments that end at site k: (s, s + 1) with k = s + 1, or the single last site of an odd span
        for (size_t g = 0; g < groups.size(); ++g) {
            const Span& z0 = sp[groups[g][0]];
            if (k < z0.i || k > z0.j) continue;
            const int s0 = z0.i + ((k - z0.i) / 2) * 2;
            if (!(k == s0 + 1 || (k == s0 && k == z0.j))) continue;
            const size_t segi = static_cast<size_t>((s0 - z0.i) / 2);
            std::ostringstream idx;
            idx << "((unsigned)q" << s0 << " * " << S->d[s0] << "u + (unsigned)n" << s0 << ")";
            if (k == s0 + 1) idx << " * " << S->d[k] << "u + (unsigned)n" << k;
            const std::string c0 = std::to_string(groups[g][0]);
            if (groups[g].size() == 2) {
                const std::string c1 = std::to_string(groups[g][1]);
                body << "    { const U2 t = *(const U2*)&SEG[" << gso[g][segi] << "u + 2u * (" << idx.str() << ")]; e" << c0
                     << " += t.x; e" << c1 << " += t.y; }\n";
            } else {
                body << "    e" << c0 << " += SEG[" << gso[g][segi] << "u + " << idx.str() << "];\n";
            }
        }
        // gathers of the channels whose span ends at site k
        for (int c = 0; c < nch; ++c) {
            if (sp[c].j != k) continue;
            const DevChan& ch = S->chans[c];
            const std::string u = std::to_string(c);
            body << "    const unsigned x" << u << " = (unsigned)n" << ch.a << " * " << S->d[ch.b] << "u + (unsigned)n" << ch.b
                 << ";\n";
            if (sp[c].j == sp[c].i + 1) {
                body << "    const C s" << u << " = LD(xs, rb + e" << u << ");\n";
            } else {
                body << "    const bool k" << u << " = (unsigned)(n" << ch.a << " - (" << ch.qa << ")) < " << S->d[ch.a]
                     << "u && (unsigned)(n" << ch.b << " - (" << ch.qb << ")) < " << S->d[ch.b] << "u;\n"
                     << "    const C s" << u << " = LD(xs, k" << u << " ? rb + e" << u << " : OOB);\n";
            }
            pending.push_back(c);
            if (static_cast<int>(pending.size()) >= kGroup) flush(false);
        }
    }
    flush(true);
    body << "    ar += dr * xf.x - di * xf.y;\n"
         << "    ai += dr * xf.y + di * xf.x;\n";
    std::ostringstream o;
    o << "// generated sector kernel: " << N << " sites, digit sum " << Q << ", " << S->Dr << " packed states, " << ndg
      << " diagonal terms in " << dkeys.size() << " tables, " << nch << " channels in " << groups.size()
      << " span groups, " << seg.size() << " rank-change table entries\n";
    if (f32)
        o << "typedef float R;\ntypedef float C __attribute__((ext_vector_type(2)));\n"
          << "typedef unsigned U __attribute__((ext_vector_type(2)));\n"
          << "#define LD(rs, vo) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64((rs), (int)(vo), 0, 0))\n"
          << "#define ST(v, rs, vo) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, (v)), (rs), (int)(vo), 0, 2)\n";
    else
        o << "typedef double R;\ntypedef double C __attribute__((ext_vector_type(2)));\n"
          << "typedef unsigned U __attribute__((ext_vector_type(4)));\n"
          << "#define LD(rs, vo) __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128((rs), (int)(vo), 0, 0))\n"
          << "#define ST(v, rs, vo) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, (v)), (rs), (int)(vo), 0, 2)\n";
    o << "typedef unsigned U2 __attribute__((ext_vector_type(2)));\n"
      << "#define OOB 0x80000000u\n"
      << "#ifndef MRMF_GROUP_FENCE\n"
      << "#define MRMF_GROUP_FENCE(a, b) __asm__ __volatile__(\"\" : \"+v\"(a), \"+v\"(b) : : \"memory\")\n"
      << "#endif\n";
    o << "__constant__ unsigned SEGC[" << std::max<size_t>(1, seg.size()) << "] = {";
    if (seg.empty()) o << "0u";
    for (size_t k = 0; k < seg.size(); ++k) o << (k ? ", " : "") << seg[k] << "u";
    o << "};\n";
    auto arr = [&](const char* ty, const char* nm, size_t n, const std::function<std::string(size_t)>& f) {
        o << "__constant__ " << ty << " " << nm << "[" << std::max<size_t>(1, n) << "] = {";
        if (n == 0) o << "0";
        for (size_t k = 0; k < n; ++k) o << (k ? ", " : "") << f(k);
        o << "};\n";
    };
    arr("int", "CB", cb.size(), [&](size_t k) { return std::to_string(cb[k]); });
    arr("int", "CP", cp.size(), [&](size_t k) { return std::to_string(cp[k]); });
    arr("R", "CVR", cvr.size(), [&](size_t k) { return lit(cvr[k], f32); });
    if (cplx) arr("R", "CVI", cvi.size(), [&](size_t k) { return lit(cvi[k], f32); });
    const size_t nseg = std::max<size_t>(2, seg.size() + (seg.size() % 2));
    // Chebyshev-step epilogue (time propagation in the sector): instead of y = H x the kernel computes
    // p = ea (H x) + eb x + eg y, writes it to y and adds (ecr + i eci) p to acc, row by row
    if (epi)
        o << "extern \"C\" __global__ __launch_bounds__(256) void mrmf_sector_cheb(const R* __restrict__ theta,\n"
          << "    const C* __restrict__ x, C* __restrict__ y, C* __restrict__ acc, R ea, R eb, R eg, R ecr, R eci,\n"
          << "    const int* __restrict__ skip, const void* __restrict__ lab) {\n";
    else
        o << "extern \"C\" __global__ __launch_bounds__(256) void mrmf_sector(const R* __restrict__ theta,\n"
          << "    const C* __restrict__ x, C* __restrict__ y, const int* __restrict__ skip, const void* __restrict__ lab) {\n";
    o << "  if (skip != nullptr && *skip != 0) return;\n"
      << "  __shared__ __attribute__((aligned(16))) unsigned SEG[" << nseg << "];\n"
      << "  for (unsigned k = threadIdx.x; k < " << seg.size() << "u; k += 256u) SEG[k] = SEGC[k];\n"
      << "  __shared__ R Tr[" << NE << "];\n";
    if (cplx) o << "  __shared__ R Ti[" << NE << "];\n";
    o << "  for (unsigned k = threadIdx.x; k < " << ent.size() << "u; k += 256u) {\n"
      << "    R sr = (R)0, si = (R)0;\n"
      << "    for (int u = CB[k]; u < CB[k + 1u]; ++u) { const R th = theta[CP[u]]; sr += th * CVR[u];"
      << (cplx ? " si += th * CVI[u];" : "") << " }\n"
      << "    Tr[k] = sr;" << (cplx ? " Ti[k] = si;" : "") << "\n"
      << "  }\n"
      << "  __syncthreads();\n"
      << "  const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, " << S->Dr * SZ
      << ", 0x00020000);\n"
      << "  const __amdgpu_buffer_rsrc_t ys = __builtin_amdgcn_make_buffer_rsrc((void*)y, (short)0, " << S->Dr * SZ
      << ", 0x00020000);\n"
      << "  const __amdgpu_buffer_rsrc_t ls = __builtin_amdgcn_make_buffer_rsrc((void*)lab, (short)0, "
      << S->Dr * S->lab_bytes << ", 0x00020000);\n";
    if (epi)
        o << "  const __amdgpu_buffer_rsrc_t as = __builtin_amdgcn_make_buffer_rsrc((void*)acc, (short)0, " << S->Dr * SZ
          << ", 0x00020000);\n";
    o
      << "  const unsigned G = gridDim.x, bk = blockIdx.x;\n";
    const int64_t ng = (S->Dr + 255) / 256;  // row groups of 256
    if (S->sched == MRMF_SCHED_XCD_CHUNK) {
        // XCD x (= block mod 8) sweeps the contiguous x-th eighth of the row groups with its blocks side by side
        o << "  const unsigned nx = (G % 8u == 0u) ? 8u : 1u, GX = G / nx, xcd = bk % nx;\n"
          << "  const unsigned Cx = (" << ng << "u + nx - 1u) / nx;\n"
          << "  const unsigned g_end = (xcd + 1u) * Cx < " << ng << "u ? (xcd + 1u) * Cx : " << ng << "u;\n"
          << "  for (unsigned g = xcd * Cx + bk / nx; g < g_end; g += GX) {\n"
          << "    const unsigned r = g * 256u + threadIdx.x;\n"
          << "    if (r >= " << S->Dr << "u) break;\n";
    } else if (S->sched == MRMF_SCHED_BLOCK_RUN) {
        // every block sweeps its own contiguous run of row groups (the runs of one XCD adjacent)
        o << "  const unsigned v = (G % 8u == 0u) ? (bk % 8u) * (G / 8u) + bk / 8u : bk;\n"
          << "  const unsigned g_end = (unsigned)(((unsigned long long)(v + 1u) * " << ng << "ull) / G);\n"
          << "  for (unsigned g = (unsigned)(((unsigned long long)v * " << ng << "ull) / G); g < g_end; ++g) {\n"
          << "    const unsigned r = g * 256u + threadIdx.x;\n"
          << "    if (r >= " << S->Dr << "u) break;\n";
    } else {
        // windows of G row groups: the blocks of one XCD (block b runs on XCD b mod 8) take one eighth of each
        // window side by side, so the rows near a channel's source were just read through that XCD's L2
        o << "  const unsigned v = (G % 8u == 0u) ? (bk % 8u) * (G / 8u) + bk / 8u : bk;\n"
          << "  for (unsigned r = v * 256u + threadIdx.x; r < " << S->Dr << "u; r += G * 256u) {\n";
    }
    o << body.str();
    if (epi)
        o << "    { const C pv = LD(ys, rb), av = LD(as, rb);\n"
          << "      C np; np.x = ea * ar + eb * xf.x + eg * pv.x; np.y = ea * ai + eb * xf.y + eg * pv.y;\n"
          << "      ST(np, ys, rb);\n"
          << "      C na; na.x = av.x + ecr * np.x - eci * np.y; na.y = av.y + ecr * np.y + eci * np.x;\n"
          << "      ST(na, as, rb); }\n";
    else
        o << "    { C out; out.x = ar; out.y = ai; ST(out, ys, rb); }\n";
    o << "  }\n}\n";
    return o.str();
}

std::string spec_source(const mrmf_plan_t* p, int dtype, Tile* tl_out, bool epi) {
    const bool f32 = dtype == MRMF_DTYPE_C;
    const int64_t SZ = f32 ? 8 : 16;
    Tile tl;
    const KernelCfg& cfg = p->cfg[epi && p->cheb_shape_set ? kSlotCheb : f32 ? MRMF_DTYPE_C : MRMF_DTYPE_Z];
    if (!choose_tiling(p, cfg.inner, cfg.unroll, cfg.unroll_top, &tl)) return "";
    const int64_t n_st = p->D / (tl.T_in * tl.P_U);
    // span of one super-tile's rows from its base (its copies of site 0 lie M_0 apart)
    int64_t st = tl.T_in * tl.P_C;
    for (int s = 0; s < tl.n_top; ++s) st += (p->d[s] - 1) * p->M[s];
    if (tl.n_top == 0) st = tl.T_in * tl.P_U;
    int64_t dmax = 0, dmin = 0;
    for (const auto& c : p->chans) {
        dmax = std::max<int64_t>(dmax, c.delta);
        dmin = std::min<int64_t>(dmin, c.delta);
    }
    // 32-bit buffer offsets when every offset (rows plus both shifts) stays below 2^31 bytes, else 64-bit
    // super-tile bases; in both forms a channel's offset from its super-tile, |Delta| + st rows, is a
    // 32-bit signed scalar
    const int64_t lim = int64_t(1) << 31;
    if (n_st >= lim || (std::max<int64_t>(dmax, -dmin) + st) * SZ >= lim) return "";
    const bool wide = cfg.wide != 0 || (p->D + dmax - dmin + 2 * tl.T_in) * SZ >= lim;
    Gen gen{p, f32, tl, static_cast<int>(round_up(tl.T_in, 64)), n_st};
    gen.wide = wide;
    gen.epi = epi;
    gen.waves_per_eu = cfg.waves_per_eu;
    gen.far_nt = cfg.far_nt;
    gen.far_dir = cfg.far_dir;
    gen.outer_first = cfg.outer_first;
    gen.sched = cfg.sched;
    gen.bskip = cfg.bskip != 0;
    gen.gs = cfg.group;
    gen.variant = cfg.variant;
    *tl_out = tl;
    if (gen.variant != MRMF_VARIANT_LIST && gen.masked_fits()) return gen.source();
    return gen.source_v2();
}

namespace {

// Compiles a generated source with hiprtc for the current device's architecture and loads kernel `name`;
// on a compile error the log (and the source) goes to *log and the result is MRMF_E_UNSUPPORTED.
mrmf_status rtc_build(const std::string& src, const char* name, const hipDeviceProp_t& prop, hipModule_t* mod_out,
                      hipFunction_t* fn_out, std::string* log_out) {
    std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mrmf_gen.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return MRMF_E_HIP;
    const char* opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult cr = hiprtcCompileProgram(prog, 7, opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string log(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &log[0]);
    if (cr != HIPRTC_SUCCESS) {
        *log_out = "hiprtc: " + log + "\n" + src;
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
    if (hipModuleGetFunction(&fn, mod, name) != hipSuccess) {
        hipModuleUnload(mod);
        return MRMF_E_HIP;
    }
    *mod_out = mod;
    *fn_out = fn;
    return MRMF_OK;
}

// slot: MRMF_DTYPE_Z, MRMF_DTYPE_C, or kSlotCheb (c128 with the Chebyshev-step epilogue)
mrmf_status compile_spec(mrmf_plan_t* p, int slot, SpecKernel& K) {
    K.tried = true;
    K.ok = false;
    const int dtype = slot == kSlotCheb ? MRMF_DTYPE_Z : slot;
    Tile tl;
    const std::string src = spec_source(p, dtype, &tl, slot == kSlotCheb);
    if (src.empty()) {
        K.log = "plan does not qualify for the specialized kernel";
        return MRMF_E_UNSUPPORTED;
    }
    const int64_t n_st = p->D / (tl.T_in * tl.P_U);
    const int block = static_cast<int>(round_up(tl.T_in, 64));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MRMF_E_HIP;
    hipModule_t mod;
    hipFunction_t fn;
    const mrmf_status bs = rtc_build(src, slot == kSlotCheb ? "mrmf_spec_cheb" : "mrmf_spec", prop, &mod, &fn, &K.log);
    if (bs != MRMF_OK) return bs;
    int per_cu = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int bpc = p->cfg[slot == kSlotCheb && p->cheb_shape_set ? kSlotCheb : dtype].blocks_per_cu;
    if (bpc > 0 && bpc < per_cu) per_cu = bpc;
    int64_t grid = int64_t(per_cu) * prop.multiProcessorCount;
    if (grid > n_st) grid = n_st;
    if (grid >= 8) grid -= grid % 8;
    K.mod = mod;
    K.fn = fn;
    K.k_in = tl.k_in;
    K.k_u = tl.k_u;
    K.T_in = static_cast<int32_t>(tl.T_in);
    K.P_U = static_cast<int32_t>(tl.P_U);
    K.block = block;
    K.grid = static_cast<int32_t>(grid);
    K.n_tiles = n_st;
    K.device = dev;
    K.log = src;
    K.ok = true;
    return MRMF_OK;
}

}  // namespace

mrmf_status spec_prepare(mrmf_plan_t* p, int dtype) {
    if (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != kSlotCheb) return MRMF_E_INVALID_ARG;
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

mrmf_status spec_launch_cheb(mrmf_plan_t* p, const double* theta, const void* x, void* prev, void* acc, double ea,
                             double eb, double eg, double ecr, double eci, hipStream_t s) {
    mrmf_status st = spec_prepare(p, kSlotCheb);
    if (st != MRMF_OK) return st;
    const SpecKernel& K = p->spec[kSlotCheb];
    struct {
        const void* theta;
        const void* x;
        void* y;
        void* acc;
        double ea, eb, eg, ecr, eci;
        const int32_t* skip;
    } args{theta, x, prev, acc, ea, eb, eg, ecr, eci, nullptr};
    size_t size = sizeof(args);
    void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size, HIP_LAUNCH_PARAM_END};
    return hip_status(hipModuleLaunchKernel(K.fn, K.grid, 1, 1, K.block, 1, 1, 0, s, nullptr, config));
}

mrmf_status grad_prepare(mrmf_plan_t* p) {
    std::lock_guard<std::mutex> lk(p->mtx);
    SpecKernel& K = p->grad;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    if (K.tried && K.device == dev) return K.ok ? MRMF_OK : MRMF_E_UNSUPPORTED;
    if (K.mod) hipModuleUnload(K.mod);
    K = SpecKernel{};
    K.device = dev;
    K.tried = true;
    const std::string src = grad_source(p);
    if (src.empty()) {
        K.log = "plan does not qualify for the generated gradient kernel";
        return MRMF_E_UNSUPPORTED;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MRMF_E_HIP;
    hipModule_t mod;
    hipFunction_t fn;
    const mrmf_status bs = rtc_build(src, "mrmf_grad", prop, &mod, &fn, &K.log);
    if (bs != MRMF_OK) return bs;
    // rows per thread against waves per SIMD: blocks_per_cu blocks of four waves on every CU (a tuning
    // knob, 2 by default), never more blocks than row groups of 256
    const int bpc = p->cfg[MRMF_DTYPE_Z].grad_blocks_per_cu > 0 ? p->cfg[MRMF_DTYPE_Z].grad_blocks_per_cu : 2;
    const int64_t groups = (p->D + 255) / 256;
    K.mod = mod;
    K.fn = fn;
    K.block = 256;
    K.grid = static_cast<int32_t>(std::min<int64_t>(groups, int64_t(bpc) * prop.multiProcessorCount));
    K.log = src;
    K.ok = true;
    return MRMF_OK;
}

bool grad_built(mrmf_plan_t* p) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(p->mtx);
    return p->grad.tried && p->grad.ok && p->grad.device == dev;
}

mrmf_status grad_launch(mrmf_plan_t* p, const double* theta, const void* x, const void* g, void* gx, double* partial,
                        int max_grid, int* grid, hipStream_t s) {
    mrmf_status st = grad_prepare(p);
    if (st != MRMF_OK) return st;
    const SpecKernel& K = p->grad;
    *grid = std::min(K.grid, max_grid);
    struct {
        const double* theta;
        const void* x;
        const void* g;
        void* gx;
        double* partial;
    } args{theta, x, g, gx, partial};
    size_t size = sizeof(args);
    void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size, HIP_LAUNCH_PARAM_END};
    return hip_status(hipModuleLaunchKernel(K.fn, *grid, 1, 1, K.block, 1, 1, 0, s, nullptr, config));
}

mrmf_status sector_gen_prepare(mrmf_sector_t* S, int slot) {
    if (slot != MRMF_DTYPE_Z && slot != MRMF_DTYPE_C && slot != kSectorSlotCheb) return MRMF_E_INVALID_ARG;
    const bool epi = slot == kSectorSlotCheb;
    std::lock_guard<std::mutex> lk(S->mtx);
    SpecKernel& K = S->gen[slot];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MRMF_E_HIP;
    if (K.tried && K.device == dev) return K.ok ? MRMF_OK : MRMF_E_UNSUPPORTED;
    if (K.mod) hipModuleUnload(K.mod);
    K = SpecKernel{};
    K.device = dev;
    K.tried = true;
    const std::string src = sector_source(S, epi ? MRMF_DTYPE_Z : slot, epi);
    if (src.empty()) {
        K.log = "sector does not qualify for the generated kernel";
        return MRMF_E_UNSUPPORTED;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MRMF_E_HIP;
    hipModule_t mod;
    hipFunction_t fn;
    const mrmf_status bs = rtc_build(src, epi ? "mrmf_sector_cheb" : "mrmf_sector", prop, &mod, &fn, &K.log);
    if (bs != MRMF_OK) return bs;
    int per_cu = S->blocks_per_cu;
    if (per_cu <= 0 &&
        (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1))
        per_cu = 1;
    const int64_t groups = (S->Dr + 255) / 256;
    K.mod = mod;
    K.fn = fn;
    K.block = 256;
    K.grid = static_cast<int32_t>(std::min<int64_t>(groups, int64_t(per_cu) * prop.multiProcessorCount));
    K.log = src;
    K.ok = true;
    return MRMF_OK;
}

mrmf_status sector_gen_launch(mrmf_sector_t* S, int dtype, const void* lab, const void* theta, const void* x, void* y,
                              hipStream_t s, const int32_t* d_skip) {
    mrmf_status st = sector_gen_prepare(S, dtype);
    if (st != MRMF_OK) return st;
    const SpecKernel& K = S->gen[dtype];
    struct {
        const void* theta;
        const void* x;
        void* y;
        const int32_t* skip;
        const void* lab;
    } args{theta, x, y, d_skip, lab};
    size_t size = sizeof(args);
    void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size, HIP_LAUNCH_PARAM_END};
    return hip_status(hipModuleLaunchKernel(K.fn, K.grid, 1, 1, K.block, 1, 1, 0, s, nullptr, config));
}

mrmf_status sector_gen_launch_cheb(mrmf_sector_t* S, const void* lab, const double* theta, const void* x, void* prev,
                                   void* acc, double ea, double eb, double eg, double ecr, double eci, hipStream_t s) {
    mrmf_status st = sector_gen_prepare(S, kSectorSlotCheb);
    if (st != MRMF_OK) return st;
    const SpecKernel& K = S->gen[kSectorSlotCheb];
    struct {
        const void* theta;
        const void* x;
        void* y;
        void* acc;
        double ea, eb, eg, ecr, eci;
        const int32_t* skip;
        const void* lab;
    } args{theta, x, prev, acc, ea, eb, eg, ecr, eci, nullptr, lab};
    size_t size = sizeof(args);
    void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &args, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size, HIP_LAUNCH_PARAM_END};
    return hip_status(hipModuleLaunchKernel(K.fn, K.grid, 1, 1, K.block, 1, 1, 0, s, nullptr, config));
}

}  // namespace mrmf

mrmf_sector_t::~mrmf_sector_t() {
    for (auto& k : gen)
        if (k.mod) hipModuleUnload(k.mod);
}

mrmf_plan_t::~mrmf_plan_t() {
    for (auto& k : spec)
        if (k.mod) hipModuleUnload(k.mod);
    if (grad.mod) hipModuleUnload(grad.mod);
}

extern "C" {

}  // extern "C"

namespace {

// Replace the kernel configuration of one element type (or of the Chebyshev-step kernel, slot
// kSlotCheb); a changed configuration drops the kernels built from it so the next call regenerates them.
// Caller holds the plan mutex.
void set_cfg(mrmf_plan_t* plan, int slot, const mrmf::KernelCfg& c) {
    mrmf::KernelCfg& cur = plan->cfg[slot];
    const bool same = cur.inner == c.inner && cur.unroll == c.unroll && cur.sched == c.sched && cur.bskip == c.bskip &&
                      cur.group == c.group && cur.blocks_per_cu == c.blocks_per_cu && cur.variant == c.variant &&
                      cur.wide == c.wide && cur.waves_per_eu == c.waves_per_eu && cur.far_nt == c.far_nt && cur.far_dir == c.far_dir &&
                      cur.outer_first == c.outer_first && cur.unroll_top == c.unroll_top &&
                      (slot != mrmf::kSlotCheb || plan->cheb_shape_set);
    cur = c;
    if (slot == mrmf::kSlotCheb) plan->cheb_shape_set = true;
    if (!same) {
        const bool cheb_follows = slot == MRMF_DTYPE_Z && !plan->cheb_shape_set;
        for (int s : {slot, cheb_follows ? mrmf::kSlotCheb : -1}) {
            if (s < 0) continue;
            mrmf::SpecKernel& k = plan->spec[s];
            if (k.mod) hipModuleUnload(k.mod);
            k = mrmf::SpecKernel{};
        }
    }
}

}  // namespace

extern "C" {

mrmf_status mrmf_plan_set_kernel(mrmf_plan plan, int32_t kind, int32_t inner_sites, int32_t unrolled_sites) {
    if (!plan || kind < MRMF_KERNEL_AUTO || kind > MRMF_KERNEL_SPECIALIZED || inner_sites < 0 ||
        inner_sites > plan->N || unrolled_sites < -1 || unrolled_sites > plan->N)
        return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mtx);
    for (int dt = 0; dt < 2; ++dt) {
        mrmf::KernelCfg c = plan->cfg[dt];
        c.mode = kind;
        c.inner = inner_sites;
        c.unroll = unrolled_sites;
        set_cfg(plan, dt, c);
    }
    return MRMF_OK;
}

mrmf_status mrmf_plan_set_tuning(mrmf_plan plan, int32_t knob, int32_t value) {
    if (!plan) return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mtx);
    for (int dt = 0; dt < 2; ++dt) {
        mrmf::KernelCfg c = plan->cfg[dt];
        switch (knob) {
            case MRMF_TUNE_SCHEDULE:
                if (value != MRMF_SCHED_WINDOWS && value != MRMF_SCHED_XCD_CHUNK && value != MRMF_SCHED_BLOCK_RUN)
                    return MRMF_E_INVALID_ARG;
                c.sched = value;
                break;
            case MRMF_TUNE_BRANCH_SKIP:
                if (value != 0 && value != 1) return MRMF_E_INVALID_ARG;
                c.bskip = value;
                break;
            case MRMF_TUNE_LOAD_GROUP:
                if (value < 0 || value > 64) return MRMF_E_INVALID_ARG;
                c.group = value;
                break;
            case MRMF_TUNE_BLOCKS_PER_CU:
                if (value < 0 || value > 32) return MRMF_E_INVALID_ARG;
                c.blocks_per_cu = value;
                break;
            case MRMF_TUNE_VARIANT:
                if (value != MRMF_VARIANT_MASKED && value != MRMF_VARIANT_LIST) return MRMF_E_INVALID_ARG;
                c.variant = value;
                break;
            case MRMF_TUNE_ADDRESSING:
                if (value != 0 && value != 1) return MRMF_E_INVALID_ARG;
                c.wide = value;
                break;
            case MRMF_TUNE_CHEB_FUSED:
                if (value != 0 && value != 1) return MRMF_E_INVALID_ARG;
                c.cheb_fused = value;
                break;
            case MRMF_TUNE_CHEB_MERGE:
                if (value != 0 && value != 1) return MRMF_E_INVALID_ARG;
                c.cheb_merge = value;
                break;
            case MRMF_TUNE_WAVES_PER_EU:
                if (value < 0 || value > 8) return MRMF_E_INVALID_ARG;
                c.waves_per_eu = value;
                break;
            case MRMF_TUNE_FAR_LOADS:
                if (value != 0 && (value < 10 || value > 40)) return MRMF_E_INVALID_ARG;
                c.far_nt = value;
                break;
            case MRMF_TUNE_FAR_DIR:
                if (value < 0 || value > 2) return MRMF_E_INVALID_ARG;
                c.far_dir = value;
                break;
            case MRMF_TUNE_OUTER_FIRST:
                if (value < 0 || value > 8) return MRMF_E_INVALID_ARG;
                c.outer_first = value;
                break;
            case MRMF_TUNE_UNROLL_TOP:
                if (value < 0 || value > 3) return MRMF_E_INVALID_ARG;
                c.unroll_top = value;
                break;
            case MRMF_TUNE_GRAD_BLOCKS_PER_CU:
                if (value < 0 || value > 8) return MRMF_E_INVALID_ARG;
                c.grad_blocks_per_cu = value;
                if (dt == MRMF_DTYPE_Z && plan->grad.mod) hipModuleUnload(plan->grad.mod);
                if (dt == MRMF_DTYPE_Z) plan->grad = mrmf::SpecKernel{};
                break;
            default: return MRMF_E_INVALID_ARG;
        }
        set_cfg(plan, dt, c);
    }
    return MRMF_OK;
}

mrmf_status mrmf_plan_set_shape(mrmf_plan plan, int32_t dtype, int32_t variant, int32_t inner_sites,
                                int32_t unrolled_sites, int32_t load_group, int32_t unroll_top) {
    if (!plan || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != MRMF_SOURCE_CHEB) ||
        (variant != MRMF_VARIANT_MASKED && variant != MRMF_VARIANT_LIST) || inner_sites < 0 ||
        inner_sites > plan->N || unrolled_sites < -1 || unrolled_sites > plan->N || load_group < 0 ||
        load_group > 64 || unroll_top < 0 || unroll_top > 3)
        return MRMF_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mtx);
    mrmf::KernelCfg c;  // schedule and block cap at their defaults
    c.mode = MRMF_KERNEL_AUTO;
    c.inner = inner_sites;
    c.unroll = unrolled_sites;
    c.variant = variant;
    c.group = load_group;
    c.cheb_fused = plan->cfg[dtype].cheb_fused;
    c.cheb_merge = plan->cfg[dtype].cheb_merge;
    c.wide = plan->cfg[dtype == MRMF_SOURCE_CHEB ? MRMF_DTYPE_Z : dtype].wide;
    c.far_nt = plan->cfg[dtype == MRMF_SOURCE_CHEB ? MRMF_DTYPE_Z : dtype].far_nt;
    c.far_dir = plan->cfg[dtype == MRMF_SOURCE_CHEB ? MRMF_DTYPE_Z : dtype].far_dir;
    c.outer_first = plan->cfg[dtype == MRMF_SOURCE_CHEB ? MRMF_DTYPE_Z : dtype].outer_first;
    c.unroll_top = unroll_top;
    set_cfg(plan, dtype, c);
    return MRMF_OK;
}

mrmf_status mrmf_plan_prepare(mrmf_plan plan, int32_t dtype) {
    if (!plan || (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != MRMF_SOURCE_GRAD))
        return MRMF_E_INVALID_ARG;
    if (dtype == MRMF_SOURCE_GRAD) return mrmf::grad_prepare(plan);
    const int32_t mode = plan->cfg[dtype].mode;
    if (mode == MRMF_KERNEL_GENERIC) return MRMF_OK;
    const mrmf_status st = mrmf::spec_prepare(plan, dtype);
    if (st == MRMF_E_UNSUPPORTED && mode == MRMF_KERNEL_AUTO) return MRMF_OK;
    return st;
}

mrmf_status mrmf_plan_autotune(mrmf_plan plan, int32_t dtype, const void* d_ws, const void* d_theta,
                               const void* d_x, void* d_y, mrmf_stream stream, int32_t* out) {
    using namespace mrmf;
    if (!plan || !d_ws || !d_theta || !d_x || !d_y || !out ||
        (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != MRMF_SOURCE_CHEB))
        return MRMF_E_INVALID_ARG;
    const bool cheb = dtype == MRMF_SOURCE_CHEB;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    struct Cand {
        int variant, inner, unrolled, group, top;
    };
    // inner blocks of 32..1024 rows, 0..2 unrolled sites with at most 9 copies, both forms, three chunk
    // sizes for the list form
    std::vector<Cand> cands;
    int64_t T = 1;
    for (int k = plan->N - 1; k >= 0; --k) {
        T *= plan->d[k];
        if (T > 1024) break;
        if (T < 32) continue;
        const int inner = plan->N - k;
        int64_t PU = 1;
        for (int u = 0; u <= 2 && u <= k; ++u) {
            if (u > 0) PU *= plan->d[k - u];
            if (PU > 9) break;
            // fewer super-tiles than a quarter of the CUs leaves the GPU idle (unless the whole
            // problem is that small)
            if (plan->D / (T * PU) < 64 && u > 0) break;
            cands.push_back({MRMF_VARIANT_MASKED, inner, u, 0, 0});
            for (int g : {4, 8, 12}) cands.push_back({MRMF_VARIANT_LIST, inner, u, g, 0});
            // site 0 unrolled as well, when a term joins it to a site of this tile (a ring's closing bond)
            const int k_u = k - u;
            bool wrap = false;
            for (const auto& c : plan->chans)
                wrap |= (c.a == 0 && c.b >= k_u) || (c.b == 0 && c.a >= k_u);
            int64_t PT = PU;
            for (int top = 1; wrap && top <= 2 && k_u > top; ++top) {  // sites 0..top-1 unrolled too
                PT *= plan->d[top - 1];
                if (PT > 16 || plan->D / (T * PT) < 64) break;
                cands.push_back({MRMF_VARIANT_MASKED, inner, u, 0, top});
                cands.push_back({MRMF_VARIANT_LIST, inner, u, 4, top});
            }
        }
    }
    if (cands.empty()) return MRMF_E_UNSUPPORTED;
    mrmf::KernelCfg cfg0;
    bool cheb_set0 = false;
    {
        std::lock_guard<std::mutex> lk(plan->mtx);
        cfg0 = plan->cfg[dtype];
        cheb_set0 = plan->cheb_shape_set;
    }
    auto apply = [&](const Cand& c, int32_t mode) {
        std::lock_guard<std::mutex> lk(plan->mtx);
        mrmf::KernelCfg k;
        k.mode = mode;
        k.inner = c.inner;
        k.unroll = c.unrolled;
        k.variant = c.variant;
        k.group = c.group;
        k.unroll_top = c.top;
        k.wide = plan->cfg[cheb ? MRMF_DTYPE_Z : dtype].wide;
        k.cheb_fused = plan->cfg[dtype].cheb_fused;
        k.cheb_merge = plan->cfg[dtype].cheb_merge;
        set_cfg(plan, dtype, k);
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MRMF_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return MRMF_E_HIP;
    }
    auto run = [&]() -> mrmf_status {
        if (cheb)  // prev = H x, acc += 0: the memory traffic of one Chebyshev step
            return spec_launch_cheb(plan, static_cast<const double*>(d_theta), d_x, d_y,
                                    static_cast<char*>(d_y) + size_t(plan->D) * 16, 1.0, 0.0, 0.0, 0.0, 0.0, s);
        return dtype == MRMF_DTYPE_Z
                   ? matvec_z_impl(plan, d_ws, static_cast<const double*>(d_theta), d_x, d_y, s, nullptr)
                   : matvec_c_impl(plan, d_ws, static_cast<const float*>(d_theta), d_x, d_y, s, nullptr);
    };
    float best = 0.f;
    int best_i = -1;
    mrmf_status st = MRMF_OK;
    for (size_t i = 0; i < cands.size(); ++i) {
        const Cand& c = cands[i];
        apply(c, MRMF_KERNEL_SPECIALIZED);
        if (spec_prepare(plan, dtype) != MRMF_OK) continue;  // this shape does not qualify
        st = run();
        if (st != MRMF_OK) break;
        hipEventRecord(e0, s);
        for (int r = 0; r < 3 && st == MRMF_OK; ++r) st = run();
        hipEventRecord(e1, s);
        if (st != MRMF_OK || hipEventSynchronize(e1) != hipSuccess) {
            st = st != MRMF_OK ? st : MRMF_E_HIP;
            break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (best_i < 0 || ms < best) {
            best = ms;
            best_i = static_cast<int>(i);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != MRMF_OK || best_i < 0) {
        std::lock_guard<std::mutex> lk(plan->mtx);
        set_cfg(plan, dtype, cfg0);
        if (cheb) plan->cheb_shape_set = cheb_set0;
        return st != MRMF_OK ? st : MRMF_E_UNSUPPORTED;
    }
    const Cand& c = cands[best_i];
    apply(c, MRMF_KERNEL_AUTO);
    st = spec_prepare(plan, dtype);
    out[0] = c.variant;
    out[1] = c.inner;
    out[2] = c.unrolled;
    out[3] = c.group;
    out[4] = static_cast<int32_t>(best / 3.f * 1000.f);  // microseconds per call
    out[5] = c.top;
    return st;
}

mrmf_status mrmf_plan_kernel_source(mrmf_plan plan, int32_t dtype, char* buf, size_t cap, size_t* len) {
    if (!plan || !len ||
        (dtype != MRMF_DTYPE_Z && dtype != MRMF_DTYPE_C && dtype != MRMF_SOURCE_CHEB && dtype != MRMF_SOURCE_GRAD) ||
        (cap > 0 && !buf))
        return MRMF_E_INVALID_ARG;
    mrmf::Tile tl;
    const bool cheb = dtype == MRMF_SOURCE_CHEB;
    const std::string src = dtype == MRMF_SOURCE_GRAD ? mrmf::grad_source(plan)
                                                      : mrmf::spec_source(plan, cheb ? MRMF_DTYPE_Z : dtype, &tl, cheb);
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
    const bool spec = plan->cfg[dtype].mode != MRMF_KERNEL_GENERIC && K.ok;
    out[0] = spec ? MRMF_KERNEL_SPECIALIZED : MRMF_KERNEL_GENERIC;
    out[1] = spec ? plan->N - K.k_in : 0;
    out[2] = spec ? K.T_in : 0;
    out[3] = spec ? K.block : 256;
    out[4] = spec ? K.grid : 0;
    out[5] = spec ? static_cast<int32_t>(K.n_tiles) : 0;
    out[6] = spec ? K.k_in - K.k_u : 0;
    out[7] = spec ? K.P_U : 0;
    return MRMF_OK;
}

}  // extern "C"
