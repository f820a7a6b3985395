// Host plan builder: validation, multipliers, local tables, channel list, device image.
//
// Mixed-radix indexing (Sec. III): M_k = prod_{l>k} d_l with site 0 most significant, D = prod d_l.
// Off-diagonal terms become channels with a fixed integer offset Delta = q_a M_a + q_b M_b and a
// per-digit coefficient table (Sec. IV, Eq. sourceoffset); diagonal terms (S_z, (S_z)^2, S_z S_z and
// the boson number operator) are kept apart since their source index is the target itself.
#include <cmath>
#include <cstring>
#include <complex>
#include <map>
#include <tuple>

#include "mrmf_internal.h"

using mrmf::DevChan;
using mrmf::DevDiag;
using mrmf::DevSite;

namespace {

int builtin_shift(int op) {
    switch (op) {
        case MRMF_OP_RAISE: return 1;
        case MRMF_OP_LOWER: return -1;
        case MRMF_OP_RAISE2: return 2;
        case MRMF_OP_LOWER2: return -2;
        default: return 0;
    }
}

// Digit shift q of an operator: <n|O|n'> is nonzero only for n - n' = q.
int shift_of(const mrmf_plan_t* p, int op) {
    return op >= MRMF_OP_LOCAL_BASE ? p->lshift[op - MRMF_OP_LOCAL_BASE] : builtin_shift(op);
}

// Hermiticity of every parameter group h_p = sum_{param_t = p} w_t O_a O_b (Sec. IV.A: h_- = conj(h_+);
// Eq. pairham: conj(J^{ab}) = J^{bar a bar b}), checked numerically: a group's terms are summed band by
// band, a band being (site a, shift q_a, site b, shift q_b) with the two sites in ascending order (operators
// on different sites commute), into the coefficient matrix M[n_a][n_b] of its target digits; the adjoint
// band (q -> -q) must carry M'[n_a - q_a][n_b - q_b] = conj(M[n_a][n_b]).
bool groups_hermitian(const mrmf_plan_t* p) {
    using Band = std::tuple<int, int, int, int>;
    std::vector<std::map<Band, std::vector<std::complex<double>>>> groups(p->n_params);
    std::vector<double> scale(p->n_params, 0.0);
    for (const auto& t : p->terms) {
        int sa = t.site_a, oa = t.op_a, sb = t.site_b, ob = t.site_b >= 0 ? t.op_b : MRMF_OP_Z;
        if (sb >= 0 && sb < sa) {
            std::swap(sa, sb);
            std::swap(oa, ob);
        }
        const int da = p->d[sa], db = sb >= 0 ? p->d[sb] : 1;
        const Band key(sa, shift_of(p, oa), sb, sb >= 0 ? shift_of(p, ob) : 0);
        auto& M = groups[t.param][key];
        if (M.empty()) M.assign(size_t(da) * db, 0.0);
        const std::complex<double> w(t.w_re, t.w_im);
        for (int na = 0; na < da; ++na) {
            const double fa = mrmf::local_factor_host(p, sa, oa, na);
            if (fa == 0.0) continue;
            for (int nb = 0; nb < db; ++nb) {
                const double fb = sb >= 0 ? mrmf::local_factor_host(p, sb, ob, nb) : 1.0;
                M[size_t(na) * db + nb] += w * fa * fb;
            }
        }
    }
    for (int g = 0; g < p->n_params; ++g)
        for (const auto& kv : groups[g])
            for (const auto& v : kv.second) scale[g] = std::max(scale[g], std::abs(v));
    for (int g = 0; g < p->n_params; ++g) {
        const double tol = 1e-12 * std::max(1.0, scale[g]);
        for (const auto& kv : groups[g]) {
            const int sa = std::get<0>(kv.first), qa = std::get<1>(kv.first);
            const int sb = std::get<2>(kv.first), qb = std::get<3>(kv.first);
            const int da = p->d[sa], db = sb >= 0 ? p->d[sb] : 1;
            auto it = groups[g].find(Band(sa, -qa, sb, -qb));
            for (int na = 0; na < da; ++na)
                for (int nb = 0; nb < db; ++nb) {
                    const std::complex<double> v = kv.second[size_t(na) * db + nb];
                    const int ma = na - qa, mb = nb - qb;
                    std::complex<double> u = 0.0;
                    if (ma >= 0 && ma < da && mb >= 0 && mb < db && it != groups[g].end())
                        u = it->second[size_t(ma) * db + mb];
                    else if (v == 0.0)
                        continue;
                    if (std::abs(v - std::conj(u)) > tol) return false;
                }
        }
    }
    return true;
}

}  // namespace

namespace mrmf {

// <n|O|n - q> of a local operator at target digit n, 0 where the source digit n - q is outside 0..d-1.
// up[n] = <n|R|n-1>, so R^2 at target n is up[n] up[n-1] and L^2 is up[n+1] up[n+2] (App. B).
double local_factor_host(const mrmf_plan_t* p, int site, int op, int n) {
    const int d = p->d[site], tab = p->tab[site];
    const double* val = p->val.data() + tab;
    const double* up = p->up.data() + tab;
    switch (op) {
        case MRMF_OP_Z: return val[n];
        case MRMF_OP_Z2: return val[n] * val[n];
        case MRMF_OP_RAISE: return n >= 1 ? up[n] : 0.0;
        case MRMF_OP_LOWER: return n <= d - 2 ? up[n + 1] : 0.0;
        case MRMF_OP_RAISE2: return n >= 2 ? up[n] * up[n - 1] : 0.0;
        case MRMF_OP_LOWER2: return n <= d - 3 ? up[n + 1] * up[n + 2] : 0.0;
        default: {  // general one-site operator: its table is zero where the source is out of range
            const int i = op - MRMF_OP_LOCAL_BASE;
            return p->up[p->lofs[i] + n];
        }
    }
}

}  // namespace mrmf

extern "C" {

const char* mrmf_status_string(mrmf_status s) {
    switch (s) {
        case MRMF_OK: return "ok";
        case MRMF_E_INVALID_ARG: return "invalid argument";
        case MRMF_E_OVERFLOW: return "basis dimension overflows the 62-bit index";
        case MRMF_E_NOT_HERMITIAN: return "a parameter group is not Hermitian";
        case MRMF_E_HIP: return "HIP runtime error";
        case MRMF_E_UNSUPPORTED: return "unsupported";
        case MRMF_E_WORKSPACE: return "workspace or scratch too small";
        default: return "unknown status";
    }
}

int32_t mrmf_version(void) { return 10000; }

mrmf_status mrmf_plan_create(int32_t n_sites, const mrmf_site* sites, int32_t n_terms,
                             const mrmf_term* terms, int32_t n_params, uint32_t flags,
                             mrmf_plan* out) {
    return mrmf_plan_create_ex(n_sites, sites, n_terms, terms, n_params, flags, 0, nullptr, out);
}

mrmf_status mrmf_plan_create_ex(int32_t n_sites, const mrmf_site* sites, int32_t n_terms,
                                const mrmf_term* terms, int32_t n_params, uint32_t flags, int32_t n_local,
                                const mrmf_local_op* local, mrmf_plan* out) {
    if (!out) return MRMF_E_INVALID_ARG;
    *out = nullptr;
    if (n_sites < 1 || n_sites > mrmf::kMaxSites || !sites) return MRMF_E_INVALID_ARG;
    if (n_terms < 0 || (n_terms > 0 && !terms) || n_params < 0) return MRMF_E_INVALID_ARG;
    if (n_local < 0 || n_local > 4096 || (n_local > 0 && !local)) return MRMF_E_INVALID_ARG;
    if (flags & ~MRMF_REQUIRE_HERMITIAN) return MRMF_E_INVALID_ARG;

    auto* p = new (std::nothrow) mrmf_plan_t();
    if (!p) return MRMF_E_INVALID_ARG;
    p->N = n_sites;
    p->n_params = n_params;
    p->flags = flags;
    p->kind.resize(n_sites);
    p->k.resize(n_sites);
    p->d.resize(n_sites);
    p->M.resize(n_sites);
    for (int i = 0; i < n_sites; ++i) {
        const int kind = sites[i].kind, k = sites[i].k;
        if ((kind != MRMF_SPIN && kind != MRMF_BOSON) || k < 1 || k + 1 > mrmf::kMaxDim) {
            delete p;
            return MRMF_E_INVALID_ARG;
        }
        p->kind[i] = kind;
        p->k[i] = k;
        p->d[i] = k + 1;
    }
    // multipliers and D with the single-word bound D < 2^62
    const int64_t limit = int64_t(1) << 62;
    int64_t acc = 1;
    for (int i = n_sites - 1; i >= 0; --i) {
        p->M[i] = acc;
        if (acc > limit / p->d[i]) {
            delete p;
            return MRMF_E_OVERFLOW;
        }
        acc *= p->d[i];
    }
    if (acc >= limit) {
        delete p;
        return MRMF_E_OVERFLOW;
    }
    p->D = acc;

    // general one-site operators
    for (int i = 0; i < n_local; ++i) {
        const mrmf_local_op& o = local[i];
        bool ok = o.site >= 0 && o.site < n_sites && o.values != nullptr;
        if (ok) ok = o.shift > -p->d[o.site] && o.shift < p->d[o.site];
        for (int n = 0; ok && n < p->d[o.site]; ++n) ok = std::isfinite(o.values[n]);
        if (!ok) {
            delete p;
            return MRMF_E_INVALID_ARG;
        }
        p->lsite.push_back(o.site);
        p->lshift.push_back(o.shift);
    }
    // terms: a general operator on its own site anywhere; built-in two-site factors Z, RAISE, LOWER
    auto op_ok = [&](int op, int site, bool pair) {
        if (op >= MRMF_OP_LOCAL_BASE) return op - MRMF_OP_LOCAL_BASE < n_local && p->lsite[op - MRMF_OP_LOCAL_BASE] == site;
        if (op < MRMF_OP_Z || op > MRMF_OP_LOWER2) return false;
        return !pair || op == MRMF_OP_Z || op == MRMF_OP_RAISE || op == MRMF_OP_LOWER;
    };
    p->terms.assign(terms, terms + n_terms);
    for (int t = 0; t < n_terms; ++t) {
        const mrmf_term& x = terms[t];
        const bool pair = x.site_b >= 0;
        bool ok = x.site_a >= 0 && x.site_a < n_sites && x.param >= 0 && x.param < n_params &&
                  std::isfinite(x.w_re) && std::isfinite(x.w_im);
        if (ok && pair)
            ok = x.site_b < n_sites && x.site_b != x.site_a && op_ok(x.op_a, x.site_a, true) &&
                 op_ok(x.op_b, x.site_b, true);
        else if (ok)
            ok = x.site_b == -1 && op_ok(x.op_a, x.site_a, false);
        if (!ok) {
            delete p;
            return MRMF_E_INVALID_ARG;
        }
    }

    // local tables: val[n] = m or n; up[n] = <n|R|n-1> = sqrt(n (d - n)) for a spin
    // (= sqrt(s(s+1) - m(m+1)) at source m = n - 1 - s, App. A Lambda), sqrt(n) for a boson (App. C)
    p->tab.resize(n_sites);
    for (int i = 0; i < n_sites; ++i) {
        p->tab[i] = static_cast<int32_t>(p->val.size());
        const int d = p->d[i];
        for (int n = 0; n < d; ++n) {
            if (p->kind[i] == MRMF_SPIN) {
                p->val.push_back(double(n) - 0.5 * double(p->k[i]));
                p->up.push_back(n == 0 ? 0.0 : std::sqrt(double(n) * double(d - n)));
            } else {
                p->val.push_back(double(n));
                p->up.push_back(std::sqrt(double(n)));
            }
        }
    }

    // general operators' tables after the sites' ones, zero where the source digit is out of range
    for (int i = 0; i < n_local; ++i) {
        const int d = p->d[local[i].site], q = local[i].shift;
        p->lofs.push_back(static_cast<int32_t>(p->up.size()));
        for (int n = 0; n < d; ++n) p->up.push_back(n - q >= 0 && n - q < d ? local[i].values[n] : 0.0);
    }
    p->hermitian = groups_hermitian(p);
    if ((flags & MRMF_REQUIRE_HERMITIAN) && !p->hermitian) {
        delete p;
        return MRMF_E_NOT_HERMITIAN;
    }

    // channels and diagonal terms
    for (int t = 0; t < n_terms; ++t) {
        const mrmf_term& x = terms[t];
        const int qa = shift_of(p, x.op_a), qb = x.site_b >= 0 ? shift_of(p, x.op_b) : 0;
        if (qa == 0 && qb == 0) {
            DevDiag g{};
            g.a = x.site_a;
            g.b = x.site_b;
            g.opa = x.op_a;
            g.opb = x.site_b >= 0 ? x.op_b : MRMF_OP_Z;
            g.param = x.param;
            g.term = t;
            g.wr = x.w_re;
            g.wi = x.w_im;
            p->diags.push_back(g);
        } else {
            DevChan c{};
            c.a = x.site_a;
            c.b = x.site_b;
            c.opa = x.op_a;
            c.opb = x.site_b >= 0 ? x.op_b : MRMF_OP_Z;
            c.qa = qa;
            c.qb = qb;
            c.param = x.param;
            c.term = t;
            c.delta = int64_t(qa) * p->M[x.site_a] + (x.site_b >= 0 ? int64_t(qb) * p->M[x.site_b] : 0);
            c.wr = x.w_re;
            c.wi = x.w_im;
            p->chans.push_back(c);
        }
    }

    // default tiling: the low sites whose product stays <= 1024 rows
    {
        int k_in = n_sites;
        int64_t T = 1;
        while (k_in > 0 && T * p->d[k_in - 1] <= 1024) {
            --k_in;
            T *= p->d[k_in];
        }
        p->tiling.k_in = k_in;
        p->tiling.T_in = static_cast<int32_t>(T);
    }

    // device image: [sites][channels][diagonal terms][val][up], sections 256-aligned
    using mrmf::align_up;
    size_t off = 0;
    p->off_site = off;
    off = align_up(off + sizeof(DevSite) * n_sites, 256);
    p->off_chan = off;
    off = align_up(off + sizeof(DevChan) * std::max<size_t>(1, p->chans.size()), 256);
    p->off_diag = off;
    off = align_up(off + sizeof(DevDiag) * std::max<size_t>(1, p->diags.size()), 256);
    p->off_val = off;
    off = align_up(off + sizeof(double) * p->val.size(), 256);
    p->off_up = off;
    off = align_up(off + sizeof(double) * p->up.size(), 256);
    p->off_lofs = off;
    off = align_up(off + sizeof(int32_t) * std::max<size_t>(1, p->lofs.size()), 256);
    // adjoint term list with per-term factor tables
    auto ftable = [&](int site, int op) {
        const int32_t at = static_cast<int32_t>(p->ftab.size());
        for (int n = 0; n < p->d[site]; ++n) p->ftab.push_back(mrmf::local_factor_host(p, site, op, n));
        return at;
    };
    for (const auto& g : p->diags)
        p->adj.push_back({g.a, g.b, ftable(g.a, g.opa), g.b >= 0 ? ftable(g.b, g.opb) : 0, g.param, 1, 0, g.wr, g.wi});
    for (const auto& c : p->chans)
        p->adj.push_back({c.a, c.b, ftable(c.a, c.opa), c.b >= 0 ? ftable(c.b, c.opb) : 0, c.param, 0, c.delta, c.wr,
                          c.wi});
    if (p->ftab.empty()) p->ftab.push_back(0.0);
    p->off_adj = off;
    off = align_up(off + sizeof(mrmf::AdjTerm) * std::max<size_t>(1, p->adj.size()), 256);
    p->off_ftab = off;
    off = align_up(off + sizeof(double) * p->ftab.size(), 256);
    p->ws_bytes = off;
    p->image.assign(off, 0);
    for (int i = 0; i < n_sites; ++i) {
        DevSite s{};
        s.d = p->d[i];
        s.tab = p->tab[i];
        s.kind = p->kind[i];
        s.M = p->M[i];
        s.magic = ~uint64_t(0) / uint64_t(p->d[i]) + 1;
        std::memcpy(p->image.data() + p->off_site + i * sizeof(DevSite), &s, sizeof(s));
    }
    if (!p->chans.empty())
        std::memcpy(p->image.data() + p->off_chan, p->chans.data(), sizeof(DevChan) * p->chans.size());
    if (!p->diags.empty())
        std::memcpy(p->image.data() + p->off_diag, p->diags.data(), sizeof(DevDiag) * p->diags.size());
    std::memcpy(p->image.data() + p->off_val, p->val.data(), sizeof(double) * p->val.size());
    std::memcpy(p->image.data() + p->off_up, p->up.data(), sizeof(double) * p->up.size());
    if (!p->lofs.empty())
        std::memcpy(p->image.data() + p->off_lofs, p->lofs.data(), sizeof(int32_t) * p->lofs.size());
    if (!p->adj.empty())
        std::memcpy(p->image.data() + p->off_adj, p->adj.data(), sizeof(mrmf::AdjTerm) * p->adj.size());
    std::memcpy(p->image.data() + p->off_ftab, p->ftab.data(), sizeof(double) * p->ftab.size());
    *out = p;
    return MRMF_OK;
}

void mrmf_plan_destroy(mrmf_plan plan) { delete plan; }

mrmf_status mrmf_plan_dim(mrmf_plan plan, int64_t* D) {
    if (!plan || !D) return MRMF_E_INVALID_ARG;
    *D = plan->D;
    return MRMF_OK;
}

mrmf_status mrmf_plan_n_offdiag(mrmf_plan plan, int32_t* n) {
    if (!plan || !n) return MRMF_E_INVALID_ARG;
    *n = static_cast<int32_t>(plan->chans.size());
    return MRMF_OK;
}

mrmf_status mrmf_plan_offdiag_terms(mrmf_plan plan, int32_t* out) {
    if (!plan || (!out && !plan->chans.empty())) return MRMF_E_INVALID_ARG;
    for (size_t c = 0; c < plan->chans.size(); ++c) out[c] = plan->chans[c].term;
    return MRMF_OK;
}

mrmf_status mrmf_plan_offsets(mrmf_plan plan, int64_t* out) {
    if (!plan || (!out && !plan->chans.empty())) return MRMF_E_INVALID_ARG;
    for (size_t c = 0; c < plan->chans.size(); ++c) out[c] = plan->chans[c].delta;
    return MRMF_OK;
}

mrmf_status mrmf_plan_workspace_bytes(mrmf_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = plan->ws_bytes;
    return MRMF_OK;
}

mrmf_status mrmf_plan_upload(mrmf_plan plan, void* d_ws, size_t ws_bytes, mrmf_stream stream) {
    if (!plan || !d_ws || !mrmf::aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    if (ws_bytes < plan->ws_bytes) return MRMF_E_WORKSPACE;
    return mrmf::hip_status(hipMemcpyAsync(d_ws, plan->image.data(), plan->ws_bytes,
                                           hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
