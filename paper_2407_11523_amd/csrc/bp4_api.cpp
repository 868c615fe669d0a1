// Host side of the C ABI declared in include/bp4.h: Tanner-graph construction
// and validation, the packed device image, argument checks, and kernel launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bp4.h"
#include "bp4_gather.h"
#include "bp4_internal.h"

using namespace bp4;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(BP4_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Host graph object.  Edges are numbered canonically (row-major nonzeros of H);
// message slots are numbered variable-major (each qubit's edges in increasing
// check order) so that a qubit's slots are contiguous.
struct bp4_graph {
    int32_t m = 0, n = 0, nnz = 0, max_cdeg = 0, max_vdeg = 0, nlog = 0, with_y = 0;
    int32_t css22 = 0;                           // X/Z labels only, <= 2 of each per qubit
    std::vector<int32_t> canon_chk, canon_var;   // canonical edge -> check, qubit
    int32_t cstride = kMaxCheckDeg;              // edge words per check
    std::vector<uint32_t> cedge;                 // [m][cstride]
    std::vector<uint32_t> vinfo;                 // [n]
    std::vector<uint32_t> vcanon;                // [nnz]
    std::vector<uint32_t> vchk;                  // [nnz] check of each message slot
    std::vector<uint32_t> sord, slev;            // serial order as levels (see graph_create)
    std::vector<uint32_t> vlab;                  // [n] slot labels of wide graphs
    std::vector<uint32_t> lptr, lent;            // logicals
    std::vector<uint32_t> gord, gedge;           // walk of the single-pass HBM kernel (narrow graphs)
    std::vector<int32_t> vptr;                   // [n + 1] first message slot of each qubit
    std::vector<int32_t> cpos;                   // [nnz] position of each message slot's edge in its check
    std::vector<uint32_t> sgedge;                // its gather words along the serial order sord
    // byte offsets of the sections in the device image
    size_t off_cedge = 0, off_vinfo = 0, off_vcanon = 0, off_vchk = 0, off_sord = 0, off_slev = 0, off_vlab = 0,
           off_lptr = 0, off_lent = 0, off_gord = 0, off_gedge = 0, off_sgedge = 0, bytes = 0;
    bool wide() const { return cstride > kMaxCheckDeg; }

    void layout()
    {
        size_t o = 0;
        off_cedge = o; o = align256(o + cedge.size() * 4);
        off_vinfo = o; o = align256(o + vinfo.size() * 4);
        off_vcanon = o; o = align256(o + vcanon.size() * 4);
        off_vchk = o; o = align256(o + vchk.size() * 4);
        off_sord = o; o = align256(o + sord.size() * 4);
        off_slev = o; o = align256(o + slev.size() * 4);
        off_vlab = o; o = align256(o + (vlab.empty() ? 1 : vlab.size()) * 4);
        off_lptr = o; o = align256(o + lptr.size() * 4);
        off_lent = o; o = align256(o + (lent.empty() ? 1 : lent.size()) * 4);
        off_gord = o; o = align256(o + (gord.empty() ? 1 : gord.size()) * 4);
        off_gedge = o; o = align256(o + (gedge.empty() ? 1 : gedge.size()) * 4);
        off_sgedge = o; o = align256(o + (sgedge.empty() ? 1 : sgedge.size()) * 4);
        bytes = o;
    }

    GraphView view(const void *dev) const
    {
        const char *b = static_cast<const char *>(dev);
        GraphView v;
        v.cedge = reinterpret_cast<const uint32_t *>(b + off_cedge);
        v.vinfo = reinterpret_cast<const uint32_t *>(b + off_vinfo);
        v.vcanon = reinterpret_cast<const uint32_t *>(b + off_vcanon);
        v.vchk = reinterpret_cast<const uint32_t *>(b + off_vchk);
        v.sord = reinterpret_cast<const uint32_t *>(b + off_sord);
        v.slev = reinterpret_cast<const uint32_t *>(b + off_slev);
        v.nlev = (int32_t)slev.size() - 1;
        v.vlab = reinterpret_cast<const uint32_t *>(b + off_vlab);
        v.cstride = cstride;
        v.lptr = reinterpret_cast<const uint32_t *>(b + off_lptr);
        v.lent = reinterpret_cast<const uint32_t *>(b + off_lent);
        v.m = m;
        v.n = n;
        v.nnz = nnz;
        v.nlog = nlog;
        return v;
    }

    GatherTables gather_view(const void *dev) const
    {
        const char *b = static_cast<const char *>(dev);
        GatherTables t;
        t.gord = reinterpret_cast<const uint32_t *>(b + off_gord);
        t.gedge = reinterpret_cast<const uint32_t *>(b + off_gedge);
        t.sord = reinterpret_cast<const uint32_t *>(b + off_sord);
        t.sgedge = reinterpret_cast<const uint32_t *>(b + off_sgedge);
        t.slev = reinterpret_cast<const uint32_t *>(b + off_slev);
        t.nlev = (int32_t)slev.size() - 1;
        return t;
    }
};

// Builds the walk (gord) and its gather words (gedge) of a narrow graph; xy: qubit
// coordinates [n][2] or NULL.
static void build_gather(bp4_graph *g, const int32_t *xy)
{
    const bp4::GatherWalkInput in{g->n, g->m, g->cstride, g->cedge.data(), g->vptr.data(), g->vchk.data(),
                                  g->cpos.data()};
    bp4::build_gather_walk(in, xy, g->gord, g->gedge);
}

extern "C" {

// Variants with a built unrolled forward and adjoint (EWAInit: param_t [T][1], the
// discounts; Momentum: [T][2], the steps and decays).
static int unrolled_variant(int32_t variant, const char *who)
{
    if (variant < BP4_BP || variant > BP4_AEWA) return fail(BP4_EINVAL, "%s: variant %d is not a bp4_variant", who, variant);
    if (variant != BP4_EWAINIT && variant != BP4_MOMENTUM)
        return fail(BP4_EUNSUPPORTED, "%s: the unrolled path is built for EWAInit-BP and Momentum-BP (variant %d)", who,
                    variant);
    return BP4_OK;
}

static int unrolled_check(const bp4_graph *g, const void *dev_graph, int32_t variant, int32_t T, int32_t K, float clamp,
                          int64_t shots, const float *param_t, const float *prior, const uint8_t *synd,
                          const uint8_t *err)
{
    if (!g || !dev_graph) return fail(BP4_EINVAL, "unrolled: NULL graph");
    int rc = unrolled_variant(variant, "unrolled");
    if (rc) return rc;
    if (g->wide()) return fail(BP4_EUNSUPPORTED, "unrolled: graphs with degrees above 4 are not supported");
    if (T < 1 || K < 1) return fail(BP4_EINVAL, "unrolled: T %d and ckpt_every %d must be >= 1", T, K);
    if (!(clamp > 0.0f)) return fail(BP4_EINVAL, "unrolled: llr_clamp must be > 0");
    if (shots < 1 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "unrolled: shots %lld outside [1, 2^31)", (long long)shots);
    if (!param_t || !prior || !synd || !err) return fail(BP4_EINVAL, "unrolled: NULL input");
    return BP4_OK;
}

int bp4_unrolled_sizes(const bp4_graph *g, int32_t variant, int32_t T, int32_t ckpt_every, int64_t shots,
                       size_t *saved_bytes, size_t *ws_bytes)
{
    if (!g || !saved_bytes || !ws_bytes) return fail(BP4_EINVAL, "unrolled_sizes: NULL argument");
    int rc = unrolled_variant(variant, "unrolled_sizes");
    if (rc) return rc;
    if (T < 1 || ckpt_every < 1) return fail(BP4_EINVAL, "unrolled_sizes: T and ckpt_every must be >= 1");
    if (shots < 1 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "unrolled_sizes: shots out of range");
    const UnrolledSizes z = unrolled_sizes(g->m, g->n, g->nnz, variant, T, ckpt_every, shots);
    *saved_bytes = z.saved;
    *ws_bytes = z.ws;
    return BP4_OK;
}

int bp4_unrolled_forward(const bp4_graph *g, const void *dev_graph, int32_t variant, int32_t T, int32_t ckpt_every,
                         float llr_clamp, int64_t shots, const float *param_t, const float *prior,
                         const uint8_t *synd, const uint8_t *err, double *loss, float *q_out, void *saved,
                         size_t saved_bytes, void *ws, size_t ws_bytes, void *stream)
{
    int rc = unrolled_check(g, dev_graph, variant, T, ckpt_every, llr_clamp, shots, param_t, prior, synd, err);
    if (rc) return rc;
    if (!loss || !saved || !ws) return fail(BP4_EINVAL, "unrolled_forward: NULL output or buffer");
    const UnrolledSizes z = unrolled_sizes(g->m, g->n, g->nnz, variant, T, ckpt_every, shots);
    if (saved_bytes < z.saved || ws_bytes < z.ws)
        return fail(BP4_EWORKSPACE, "unrolled_forward: saved %zu < %zu or ws %zu < %zu bytes", saved_bytes, z.saved,
                    ws_bytes, z.ws);
    hipError_t e = launch_unrolled_forward(g->view(dev_graph), variant, T, ckpt_every, llr_clamp, (int32_t)shots, param_t,
                                           prior, synd, err, loss, q_out, saved, ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "unrolled_forward: launch");
    return BP4_OK;
}

int bp4_unrolled_backward(const bp4_graph *g, const void *dev_graph, int32_t variant, int32_t T, int32_t ckpt_every,
                          float llr_clamp, int64_t shots, const float *param_t, const float *prior,
                          const uint8_t *synd, const uint8_t *err, const float *dloss, const void *saved,
                          size_t saved_bytes, double *dparam_t, double *dprior, void *ws, size_t ws_bytes,
                          void *stream)
{
    int rc = unrolled_check(g, dev_graph, variant, T, ckpt_every, llr_clamp, shots, param_t, prior, synd, err);
    if (rc) return rc;
    if (!dparam_t || !dprior || !saved || !ws) return fail(BP4_EINVAL, "unrolled_backward: NULL output or buffer");
    const UnrolledSizes z = unrolled_sizes(g->m, g->n, g->nnz, variant, T, ckpt_every, shots);
    if (saved_bytes < z.saved || ws_bytes < z.ws)
        return fail(BP4_EWORKSPACE, "unrolled_backward: saved %zu < %zu or ws %zu < %zu bytes", saved_bytes,
                    z.saved, ws_bytes, z.ws);
    hipError_t e = launch_unrolled_backward(g->view(dev_graph), variant, T, ckpt_every, llr_clamp, (int32_t)shots, param_t,
                                            prior, synd, err, dloss, saved, dparam_t, dprior, ws,
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "unrolled_backward: launch");
    return BP4_OK;
}

int bp4_prior_llr(int32_t n, const double *probs, float *prior, void *stream)
{
    if (!probs || !prior) return fail(BP4_EINVAL, "prior_llr: NULL argument");
    if (n < 1 || n > kMaxVars) return fail(BP4_EINVAL, "prior_llr: n %d outside [1, %d]", n, kMaxVars);
    hipError_t e = launch_prior_llr(n, probs, prior, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "prior_llr: launch");
    return BP4_OK;
}

const char *bp4_last_error(void) { return g_err.c_str(); }

const char *bp4_version(void) { return "bp4 0.1 gfx950"; }

int bp4_graph_create(const uint8_t *hx, const uint8_t *hz, int32_t m, int32_t n, uint32_t flags,
                     bp4_graph **out)
{
    if (!out) return fail(BP4_EINVAL, "graph_create: out is NULL");
    *out = nullptr;
    if (!hx || !hz) return fail(BP4_EINVAL, "graph_create: NULL matrix");
    if (m <= 0 || n <= 0) return fail(BP4_EINVAL, "graph_create: m=%d n=%d must be positive", m, n);
    if (n > kMaxVars) return fail(BP4_EUNSUPPORTED, "graph_create: n=%d above %d", n, kMaxVars);
    std::vector<int32_t> cdeg(m, 0), vdeg(n, 0);
    long nnz = 0;
    for (long i = 0; i < (long)m * n; ++i) {
        if (hx[i] > 1 || hz[i] > 1)
            return fail(BP4_EINVAL, "graph_create: entry (%ld,%ld) not 0/1", i / n, i % n);
        if (hx[i] | hz[i]) {
            ++cdeg[i / n];
            ++vdeg[i % n];
            ++nnz;
        }
    }
    if (nnz > kMaxEdges) return fail(BP4_EUNSUPPORTED, "graph_create: %ld edges above %d", nnz, kMaxEdges);
    int maxc = 0, maxv = 0;
    for (int c = 0; c < m; ++c) {
        if (cdeg[c] == 0) return fail(BP4_EINVAL, "graph_create: check %d is empty", c);
        maxc = cdeg[c] > maxc ? cdeg[c] : maxc;
    }
    for (int v = 0; v < n; ++v) {
        if (vdeg[v] == 0) return fail(BP4_EINVAL, "graph_create: qubit %d is in no check", v);
        maxv = vdeg[v] > maxv ? vdeg[v] : maxv;
    }
    if (maxc > kMaxCheckDegWide || maxv > kMaxVarDegWide)
        return fail(BP4_EDEGREE, "graph_create: degrees (check %d, qubit %d) above (%d, %d)", maxc, maxv,
                    kMaxCheckDegWide, kMaxVarDegWide);

    auto *g = new bp4_graph;
    g->m = m;
    g->n = n;
    g->nnz = (int32_t)nnz;
    g->max_cdeg = maxc;
    g->max_vdeg = maxv;
    g->cstride = (maxc > kMaxCheckDeg || maxv > kMaxVarDeg) ? kMaxCheckDegWide : kMaxCheckDeg;
    std::vector<uint32_t> lab(nnz);
    for (long i = 0; i < (long)m * n; ++i)
        if (hx[i] && hz[i]) g->with_y = 1;
    for (int c = 0; c < m; ++c)
        for (int v = 0; v < n; ++v) {
            const long i = (long)c * n + v;
            if (hx[i] | hz[i]) {
                g->canon_chk.push_back(c);
                g->canon_var.push_back(v);
                lab[g->canon_chk.size() - 1] = (uint32_t)(hx[i] | (hz[i] << 1));
            }
        }
    // variable-major slots
    std::vector<int32_t> vptr(n + 1, 0);
    for (int v = 0; v < n; ++v) vptr[v + 1] = vptr[v] + vdeg[v];
    std::vector<int32_t> fill(n, 0), slot_of(nnz);
    g->vcanon.assign(nnz, 0);
    for (long k = 0; k < nnz; ++k) {   // canonical order visits checks increasingly
        const int v = g->canon_var[k];
        const int s = vptr[v] + fill[v]++;
        slot_of[k] = s;
        g->vcanon[s] = (uint32_t)k;
    }
    g->vchk.assign(nnz, 0);
    for (long s = 0; s < nnz; ++s) g->vchk[s] = (uint32_t)g->canon_chk[g->vcanon[s]];
    // X/Z-only graphs with at most two edges of each label per qubit (planar, toric and
    // XZZX surface codes) take the LDS kernel's two-plus-two message layout
    if (!g->with_y && g->cstride == kMaxCheckDeg) {
        std::vector<int32_t> nx(n, 0), nz(n, 0);
        for (long k = 0; k < nnz; ++k) (lab[k] == 1u ? nx : nz)[g->canon_var[k]]++;
        g->css22 = 1;
        for (int v = 0; v < n; ++v)
            if (nx[v] > 2 || nz[v] > 2) g->css22 = 0;
    }
    // Serial order (Algorithm 1) as levels: level(v) = 1 + the largest level of an
    // earlier qubit sharing a check with v (0 if none).  Qubits of one level share
    // no check, and every neighbour of v that precedes it in index order sits on a
    // lower level, every later one on a higher level, so sweeping the levels in
    // order, each level's qubits in parallel, reads and writes exactly what the
    // qubit-by-qubit sweep does.  sord: qubits by (level, index); slev: offsets.
    std::vector<int32_t> lev(n, 0);
    {
        std::vector<int32_t> chk_top(m, -1);
        int32_t nlev = 0;
        for (int v = 0; v < n; ++v) {
            int32_t l = 0;
            for (int32_t s = vptr[v]; s < vptr[v + 1]; ++s) l = std::max(l, chk_top[g->vchk[s]] + 1);
            lev[v] = l;
            for (int32_t s = vptr[v]; s < vptr[v + 1]; ++s) chk_top[g->vchk[s]] = std::max(chk_top[g->vchk[s]], l);
            nlev = std::max(nlev, l + 1);
        }
        g->slev.assign(nlev + 1, 0);
        for (int v = 0; v < n; ++v) ++g->slev[lev[v] + 1];
        for (int l = 0; l < nlev; ++l) g->slev[l + 1] += g->slev[l];
        std::vector<uint32_t> pos(g->slev.begin(), g->slev.end() - 1);
        g->sord.assign(n, 0);
        for (int v = 0; v < n; ++v) g->sord[pos[lev[v]]++] = (uint32_t)v;
    }
    // commutation of the rows: only pairs sharing a qubit can anticommute
    if (!(flags & BP4_ALLOW_ANTICOMMUTING)) {
        std::vector<std::vector<std::pair<int, uint32_t>>> vchk(n);
        for (long k = 0; k < nnz; ++k) vchk[g->canon_var[k]].push_back({g->canon_chk[k], lab[k]});
        std::vector<int32_t> cptr(m + 1, 0);
        for (int c = 0; c < m; ++c) cptr[c + 1] = cptr[c] + cdeg[c];
        std::vector<uint8_t> par(m, 0), seen(m, 0);
        std::vector<int> touched;
        for (int c = 0; c < m; ++c) {
            touched.clear();
            for (int k = cptr[c]; k < cptr[c + 1]; ++k) {
                const uint32_t a = lab[k];
                for (auto &pr : vchk[g->canon_var[k]]) {
                    const int c2 = pr.first;
                    if (c2 <= c) continue;
                    const uint32_t b = pr.second;
                    if (!seen[c2]) { seen[c2] = 1; touched.push_back(c2); }
                    par[c2] ^= (uint8_t)(((a & (b >> 1)) ^ ((a >> 1) & b)) & 1u);
                }
            }
            for (int c2 : touched) {
                if (par[c2]) {
                    delete g;
                    return fail(BP4_ENONCOMM, "graph_create: rows %d and %d anticommute", c, c2);
                }
            }
            for (int c2 : touched) { par[c2] = 0; seen[c2] = 0; }
        }
    }
    // packed check edges (ELL, padded)
    g->cedge.assign((size_t)m * g->cstride, edge_pad_word((int)nnz));
    std::vector<int32_t> cpos_of_slot(nnz, 0);   // position of each message slot's edge in its check
    {
        std::vector<int> cfill(m, 0);
        for (long k = 0; k < nnz; ++k) {
            const int c = g->canon_chk[k];
            const uint32_t w = (uint32_t)slot_of[k] | ((uint32_t)g->canon_var[k] << 16) | (lab[k] << 30);
            cpos_of_slot[slot_of[k]] = cfill[c];
            g->cedge[(size_t)c * g->cstride + cfill[c]++] = w;
        }
    }
    // walk and gather words of the single-pass HBM kernel (narrow graphs)
    if (!g->wide()) {
        g->vptr = vptr;
        g->cpos = cpos_of_slot;
        build_gather(g, nullptr);
        // the same words along the serial order, with bit 24 + k set where the k-th other
        // position of the check belongs to a qubit on a lower level (updated earlier in the
        // same sweep)
        g->sgedge.assign((size_t)4 * n, kGatherAbsent);
        for (int i = 0; i < n; ++i) {
            const int v = (int)g->sord[i];
            for (int j = 0; j < vdeg[v]; ++j) {
                const int32_t s = vptr[v] + j;
                const uint32_t c = g->vchk[s], p = (uint32_t)cpos_of_slot[s];
                const uint32_t pad = (0xFu << cdeg[c]) & 0xFu;
                uint32_t w = (4u * c + p) | (pad << 20);
                for (uint32_t k = 0; k < 3; ++k) {
                    const uint32_t pk = k + (k >= p ? 1u : 0u);
                    const uint32_t e = g->cedge[(size_t)c * g->cstride + pk];
                    if (!edge_is_pad(e) && lev[edge_var(e)] < lev[v]) w |= 1u << (kGatherEarlierShift + k);
                }
                g->sgedge[(size_t)4 * i + j] = w;
            }
        }
    }
    // packed qubit words
    g->vinfo.assign(n, 0);
    if (g->wide()) g->vlab.assign(n, 0);
    for (int v = 0; v < n; ++v) {
        uint32_t w = (uint32_t)vptr[v] | ((uint32_t)vdeg[v] << 16);
        for (int j = 0; j < vdeg[v]; ++j) {
            const uint32_t l = lab[g->vcanon[vptr[v] + j]];
            if (g->wide())
                g->vlab[v] |= l << (2 * j);
            else
                w |= l << (20 + 2 * j);
            w |= 1u << (27 + l);
        }
        g->vinfo[v] = w;
    }
    g->lptr.assign(1, 0);
    g->layout();
    *out = g;
    return BP4_OK;
}

int bp4_graph_set_logicals(bp4_graph *g, const uint8_t *lx, const uint8_t *lz, int32_t nlog)
{
    if (!g) return fail(BP4_EINVAL, "set_logicals: NULL graph");
    if (nlog < 0 || (nlog > 0 && (!lx || !lz))) return fail(BP4_EINVAL, "set_logicals: bad arguments");
    std::vector<uint32_t> ptr(1, 0), ent;
    for (int k = 0; k < nlog; ++k) {
        for (int v = 0; v < g->n; ++v) {
            const uint8_t x = lx[(size_t)k * g->n + v], z = lz[(size_t)k * g->n + v];
            if (x > 1 || z > 1) return fail(BP4_EINVAL, "set_logicals: entry not 0/1");
            if (x | z) ent.push_back((uint32_t)v | ((uint32_t)(x | (z << 1)) << 16));
        }
        ptr.push_back((uint32_t)ent.size());
    }
    g->lptr = ptr;
    g->lent = ent;
    g->nlog = nlog;
    g->layout();
    return BP4_OK;
}

int bp4_graph_set_coords(bp4_graph *g, const int32_t *xy)
{
    if (!g || !xy) return fail(BP4_EINVAL, "set_coords: NULL argument");
    if (g->wide()) return fail(BP4_EUNSUPPORTED, "set_coords: no single-pass HBM kernel for graphs with degrees above 4");
    build_gather(g, xy);
    return BP4_OK;
}

int bp4_graph_info(const bp4_graph *g, int32_t *n, int32_t *m, int32_t *nnz, int32_t *max_cdeg,
                   int32_t *max_vdeg)
{
    if (!g) return fail(BP4_EINVAL, "graph_info: NULL graph");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (nnz) *nnz = g->nnz;
    if (max_cdeg) *max_cdeg = g->max_cdeg;
    if (max_vdeg) *max_vdeg = g->max_vdeg;
    return BP4_OK;
}

int bp4_graph_device_bytes(const bp4_graph *g, size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "graph_device_bytes: NULL argument");
    *bytes = g->bytes;
    return BP4_OK;
}

int bp4_graph_edges(const bp4_graph *g, int32_t *check, int32_t *qubit)
{
    if (!g || !check || !qubit) return fail(BP4_EINVAL, "graph_edges: NULL argument");
    std::memcpy(check, g->canon_chk.data(), sizeof(int32_t) * g->nnz);
    std::memcpy(qubit, g->canon_var.data(), sizeof(int32_t) * g->nnz);
    return BP4_OK;
}

int bp4_graph_upload(const bp4_graph *g, void *dev_buf, size_t bytes, void *stream)
{
    if (!g || !dev_buf) return fail(BP4_EINVAL, "graph_upload: NULL argument");
    if (bytes < g->bytes) return fail(BP4_EWORKSPACE, "graph_upload: %zu bytes < %zu", bytes, g->bytes);
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255) return fail(BP4_EINVAL, "graph_upload: buffer not 256-byte aligned");
    std::vector<uint8_t> img(g->bytes, 0);
    std::memcpy(img.data() + g->off_cedge, g->cedge.data(), g->cedge.size() * 4);
    std::memcpy(img.data() + g->off_vinfo, g->vinfo.data(), g->vinfo.size() * 4);
    std::memcpy(img.data() + g->off_vcanon, g->vcanon.data(), g->vcanon.size() * 4);
    std::memcpy(img.data() + g->off_vchk, g->vchk.data(), g->vchk.size() * 4);
    std::memcpy(img.data() + g->off_sord, g->sord.data(), g->sord.size() * 4);
    std::memcpy(img.data() + g->off_slev, g->slev.data(), g->slev.size() * 4);
    if (!g->vlab.empty()) std::memcpy(img.data() + g->off_vlab, g->vlab.data(), g->vlab.size() * 4);
    std::memcpy(img.data() + g->off_lptr, g->lptr.data(), g->lptr.size() * 4);
    if (!g->lent.empty()) std::memcpy(img.data() + g->off_lent, g->lent.data(), g->lent.size() * 4);
    if (!g->gord.empty()) std::memcpy(img.data() + g->off_gord, g->gord.data(), g->gord.size() * 4);
    if (!g->gedge.empty()) std::memcpy(img.data() + g->off_gedge, g->gedge.data(), g->gedge.size() * 4);
    if (!g->sgedge.empty()) std::memcpy(img.data() + g->off_sgedge, g->sgedge.data(), g->sgedge.size() * 4);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(dev_buf, img.data(), g->bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "graph_upload: hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "graph_upload: hipStreamSynchronize");
    return BP4_OK;
}

void bp4_graph_destroy(bp4_graph *g) { delete g; }

}  // extern "C"

namespace {

int check_params(const bp4_params *p)
{
    if (!p) return fail(BP4_EINVAL, "params: NULL");
    if (p->variant < BP4_BP || p->variant > BP4_AEWA) return fail(BP4_EINVAL, "params: variant %d", p->variant);
    if (p->max_iter < 1) return fail(BP4_EINVAL, "params: max_iter %d < 1", p->max_iter);
    if (!(p->llr_clamp > 0.0f) || !std::isfinite(p->llr_clamp)) return fail(BP4_EINVAL, "params: llr_clamp must be finite and > 0");
    if (p->variant == BP4_MOMENTUM || p->variant == BP4_EWAINIT || p->variant == BP4_AEWA) {
        if (!(p->alpha >= 0.0f && p->alpha <= 1.0f)) return fail(BP4_EINVAL, "params: alpha must lie in [0, 1]");
    }
    if (p->serial != 0 && p->serial != 1) return fail(BP4_EINVAL, "params: serial must be 0 or 1");
    if (p->variant == BP4_AEWA) {
        if (!(p->alpha_last >= 0.0f && p->alpha_last <= 1.0f))
            return fail(BP4_EINVAL, "params: alpha_last must lie in [0, 1]");
        if (p->alpha_steps < 1 || p->alpha_steps > 64) return fail(BP4_EINVAL, "params: alpha_steps outside [1, 64]");
        if (!p->stop_on_syndrome) return fail(BP4_EINVAL, "params: AEWA restarts on a failed syndrome test: stop_on_syndrome must be 1");
    }
    if (p->variant == BP4_MOMENTUM && !(p->gamma >= 0.0f && p->gamma < 1.0f))
        return fail(BP4_EINVAL, "params: gamma must lie in [0, 1)");
    if (p->variant == BP4_ADAGRAD) {
        if (!(p->alpha > 0.0f) || !std::isfinite(p->alpha)) return fail(BP4_EINVAL, "params: AdaGrad alpha must be > 0");
        if (!(p->eps > 0.0f) || !std::isfinite(p->eps)) return fail(BP4_EINVAL, "params: eps must be > 0");
    }
    return BP4_OK;
}

constexpr size_t kSmallWorkspace = 256;   // one queue counter, padded

// Largest dynamic LDS allocation of one workgroup on the current device.
int device_max_lds(size_t *bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    *bytes = (size_t)v;
    return BP4_OK;
}

void fill_decode_args(DecodeArgs &a, const bp4_graph *g, const void *dev_graph, const bp4_params *p,
                      int64_t shots, const float *prior_llr, const uint8_t *synd, uint8_t *est,
                      uint8_t *conv, int32_t *iters, const LdsLayout &L, unsigned int *counter)
{
    a.g = g->view(dev_graph);
    a.prior = prior_llr;
    a.synd = synd;
    a.est = est;
    a.conv = conv;
    a.iters = iters;
    a.q_out = nullptr;
    a.mvc_out = nullptr;
    a.mcv_out = nullptr;
    a.counter = counter;
    a.shots = (int32_t)shots;
    a.variant = p->variant;
    a.max_iter = p->max_iter;
    a.stop = p->stop_on_syndrome ? 1 : 0;
    a.g_from_t1 = p->adagrad_g_from_t1 ? 1 : 0;
    a.alpha = p->alpha;
    a.gamma = p->gamma;
    a.eps = p->eps;
    a.clamp = p->llr_clamp;
    a.alpha_last = p->alpha_last;
    a.alpha_steps = p->alpha_steps;
    a.static_words = L.static_words;
    a.region_words = L.region_words;
    a.q_off = L.q_off;
    a.acc_off = L.acc_off;
    a.ehat_off = L.ehat_off;
    a.syn_off = L.syn_off;
    a.hdr_off = L.hdr_off;
    a.group_lanes = L.group_lanes;
    a.block_shots = L.block_shots;
    a.magic_m = (uint32_t)(((1ull << 32) + (uint64_t)g->m - 1) / (uint64_t)g->m);
    a.magic_n = (uint32_t)(((1ull << 32) + (uint64_t)g->n - 1) / (uint64_t)g->n);
    a.with_y = g->with_y;
    a.wide = g->wide() ? 1 : 0;
    a.css22 = g->css22;
}

// The automatic kernel: SOA when even one shot per workgroup needs more than
// kLdsAutoLimit bytes of LDS, or the code has more than 64 checks per lane.
int auto_kernel(const bp4_graph *g, int variant)
{
    if (g->wide()) return BP4_KERNEL_LDS;   // the only kernel for wide graphs
    if (!decode_lds_fits(g->m, g->n, kLdsBlock, 1)) return BP4_KERNEL_SOA;
    return decode_lds_layout(g->m, g->n, g->nnz, variant, kLdsBlock, 1).bytes > kLdsAutoLimit ? BP4_KERNEL_SOA
                                                                                      : BP4_KERNEL_LDS;
}

// LDS the single-pass HBM kernel may take per workgroup (the two per-check masks):
// the 64 KB every workgroup is guaranteed.
constexpr size_t kGatherMaxLds = 65536;

bool gather_ok(const bp4_graph *g, int variant, int serial)
{
    return gather_supported(g->m, variant, serial, g->wide(), kGatherMaxLds);
}

// Large codes under AUTO: the single-pass HBM kernel where it applies (no verification
// outputs), else the two-phase SOA kernel.
int large_kernel(const bp4_graph *g, int variant, int serial, bool verify)
{
    return !verify && gather_ok(g, variant, serial) ? BP4_KERNEL_GATHER : BP4_KERNEL_SOA;
}

// Serial schedule on the LDS kernel: wave groups of G in {1, 2, 4, ..., 64} lanes.
// Lane use = the share of (lane, level pass) pairs that carry a qubit of the level.
static double serial_lane_use(const bp4_graph *g, int G)
{
    double used = 0.0, issued = 0.0;
    for (size_t l = 0; l + 1 < g->slev.size(); ++l) {
        const double w = (double)(g->slev[l + 1] - g->slev[l]);
        used += w;
        issued += G * std::ceil(w / G);
    }
    return issued > 0.0 ? used / issued : 0.0;
}

static LdsLayout serial_layout(const bp4_graph *g, int variant, int G)
{
    return decode_lds_serial_layout(g->m, g->n, g->nnz, (int)g->slev.size() - 1, variant, G, g->wide());
}

// The serial kernel the automatic choice takes: LDS when 64-lane groups fit
// kLdsAutoLimit, else the SOA kernel.
int serial_auto_kernel(const bp4_graph *g, int variant)
{
    return serial_layout(g, variant, 64).bytes > kLdsAutoLimit ? BP4_KERNEL_SOA : BP4_KERNEL_LDS;
}

int choose_serial_lanes(const bp4_graph *g, const bp4_params *p, int32_t G, int32_t S, size_t max_lds, int *out)
{
    if (S != 0) return fail(BP4_EINVAL, "decode: the serial schedule runs on wave groups (block_shots must be 0)");
    if (G != 0 && G != 1 && G != 2 && G != 4 && G != 8 && G != 16 && G != 32 && G != 64)
        return fail(BP4_EINVAL, "decode: serial group_lanes %d not in {1, 2, 4, ..., 64}", G);
    if (G) {
        if (serial_layout(g, p->variant, G).bytes > max_lds)
            return fail(BP4_EINVAL, "decode: serial group_lanes %d exceeds the LDS of a workgroup", G);
        *out = G;
        return BP4_OK;
    }
    // default: lane use over the level passes times the occupancy the LDS allows
    const double cu_lds = 160.0 * 1024.0;
    double best_score = -1.0;
    int best = -1;
    for (int c = 64; c >= 1; c /= 2) {
        const LdsLayout L = serial_layout(g, p->variant, c);
        if (L.bytes > max_lds) continue;
        double waves = std::floor(cu_lds / (double)L.bytes) * (L.block / 64);
        if (waves > 16.0) waves = 16.0;
        const double score = serial_lane_use(g, c) * waves / 16.0;
        if (score > best_score * 1.02) {
            best_score = score;
            best = c;
        }
    }
    if (best < 0) return fail(BP4_EUNSUPPORTED, "decode: code too large for the serial LDS kernel");
    *out = best;
    return BP4_OK;
}

// A requested lane mapping in range: group_lanes 0 or a power of two in
// [4, kLdsBlock]; block_shots in [0, kLdsBlock], only with group_lanes 0 or kLdsBlock.
int check_lanes(int32_t G, int32_t S, const char *who)
{
    if (G != 0 && (G < 4 || G > kLdsBlock || (G & (G - 1)) != 0))
        return fail(BP4_EINVAL, "%s: group_lanes %d not in {4, 8, ..., %d}", who, G, kLdsBlock);
    if (S < 0 || S > kLdsBlock) return fail(BP4_EINVAL, "%s: block_shots %d outside [0, %d]", who, S, kLdsBlock);
    if (S > 0 && G != 0 && G != kLdsBlock)
        return fail(BP4_EINVAL, "%s: block_shots needs group_lanes 0 or %d", who, kLdsBlock);
    return BP4_OK;
}

// Lane mapping for one code: the caller's choice (validated) or the default pick.
// group_lanes 128, 256 and 512 are block slots with 4, 2 and 1 shots per workgroup.
int choose_lanes(const bp4_graph *g, const bp4_params *p, int32_t G, int32_t S, size_t max_lds, LaneChoice *out,
                 int64_t shots = 0)
{
    int rc = check_lanes(G, S, "decode");
    if (rc) return rc;
    if (G == 0 && S == 0) {
        *out = decode_lds_pick(g->m, g->n, g->nnz, p->variant, max_lds, g->wide(), shots);
        if (out->group_lanes < 0) return fail(BP4_EUNSUPPORTED, "decode: code too large for the LDS kernel");
        return BP4_OK;
    }
    if (G > 64 || S > 0) {
        if (S == 0) S = kLdsBlock / G;
        G = kLdsBlock;
    }
    if (!decode_lds_fits(g->m, g->n, G, S))
        return fail(BP4_EINVAL, "decode: %d lanes x %d shots leave more than 64 checks per lane", G, S);
    if (decode_lds_layout(g->m, g->n, g->nnz, p->variant, G, S, g->wide()).bytes > max_lds)
        return fail(BP4_EINVAL, "decode: group_lanes %d, block_shots %d exceed the LDS of a workgroup", G, S);
    out->group_lanes = G;
    out->block_shots = S;
    return BP4_OK;
}

int decode_common(const bp4_graph *g, const void *dev_graph, const bp4_params *p,
                  const bp4_tuning *tune, int64_t shots,
                  const float *prior_llr, const uint8_t *synd, uint8_t *est, uint8_t *conv,
                  int32_t *iters, float *q_out, float *mvc_out, float *mcv_out, void *ws,
                  size_t ws_bytes, void *stream)
{
    if (!g || !dev_graph) return fail(BP4_EINVAL, "decode: NULL graph");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "decode: shots %lld outside [0, 2^31)", (long long)shots);
    if (!prior_llr) return fail(BP4_EINVAL, "decode: NULL prior");
    if (shots == 0) return BP4_OK;
    if (!synd || !est || !conv || !iters) return fail(BP4_EINVAL, "decode: NULL buffer");
    if ((mvc_out == nullptr) != (mcv_out == nullptr)) return fail(BP4_EINVAL, "decode: mvc_out and mcv_out go together");
    if (!ws) return fail(BP4_EINVAL, "decode: NULL workspace");
    if (ws_bytes < kSmallWorkspace) return fail(BP4_EWORKSPACE, "decode: workspace %zu < %zu bytes", ws_bytes, kSmallWorkspace);
    int32_t requested = 0, requested_S = 0, lds_floor = 0, kernel = BP4_KERNEL_AUTO, soa_lanes = 0, soa_block = 0;
    int32_t gather_waves = 0;
    if (tune) {
        if (tune->reserved) return fail(BP4_EINVAL, "decode: reserved tuning fields must be 0");
        lds_floor = tune->lds_bytes;
        if (lds_floor < 0) return fail(BP4_EINVAL, "decode: negative lds_bytes");
        kernel = tune->kernel;
        if (kernel != BP4_KERNEL_AUTO && kernel != BP4_KERNEL_LDS && kernel != BP4_KERNEL_SOA &&
            kernel != BP4_KERNEL_GATHER)
            return fail(BP4_EINVAL, "decode: kernel %d unknown", kernel);
        soa_lanes = tune->soa_lanes;
        soa_block = tune->soa_iter_block;
        if (soa_lanes < 0 || soa_block < 0) return fail(BP4_EINVAL, "decode: negative soa_lanes or soa_iter_block");
        gather_waves = tune->gather_waves;
        if (gather_waves != 0 && gather_waves != 4 && gather_waves != 8 && gather_waves != 16)
            return fail(BP4_EINVAL, "decode: gather_waves %d not 0, 4, 8 or 16", gather_waves);
        requested = tune->group_lanes;
        requested_S = tune->block_shots;
        if (!p->serial) {
            rc = check_lanes(requested, requested_S, "decode");
            if (rc) return rc;
        }
    }
    const bool lds_knobs = requested || requested_S || lds_floor, soa_knobs = soa_lanes || soa_block;
    const bool gather_knobs = gather_waves != 0, verify = q_out || mvc_out;
    if ((int)lds_knobs + (int)soa_knobs + (int)gather_knobs > 1)
        return fail(BP4_EINVAL, "decode: LDS, SOA and gather tuning fields exclude each other");
    if (kernel == BP4_KERNEL_AUTO) {
        kernel = lds_knobs ? BP4_KERNEL_LDS
                 : soa_knobs ? BP4_KERNEL_SOA
                 : gather_knobs ? BP4_KERNEL_GATHER
                 : p->serial ? serial_auto_kernel(g, p->variant) : auto_kernel(g, p->variant);
        if (kernel == BP4_KERNEL_SOA && !soa_knobs) kernel = large_kernel(g, p->variant, p->serial, verify);
    }
    if (kernel == BP4_KERNEL_LDS && soa_knobs)
        return fail(BP4_EINVAL, "decode: soa_lanes and soa_iter_block apply to the SOA kernel");
    if (kernel != BP4_KERNEL_GATHER && gather_knobs)
        return fail(BP4_EINVAL, "decode: gather_waves applies to the single-pass HBM kernel");
    if (g->wide() && kernel != BP4_KERNEL_LDS)
        return fail(BP4_EUNSUPPORTED, "decode: graphs with degrees above 4 run the LDS kernel only");
    if (kernel == BP4_KERNEL_GATHER) {
        if (lds_knobs || soa_knobs)
            return fail(BP4_EINVAL, "decode: LDS and SOA tuning fields do not apply to the single-pass HBM kernel");
        if (!gather_ok(g, p->variant, p->serial))
            return fail(BP4_EUNSUPPORTED, "decode: the single-pass HBM kernel runs narrow codes of at most %zu checks",
                        (kGatherMaxLds - 64 * 4) / 16 - 1);
        if (verify) return fail(BP4_EUNSUPPORTED, "decode: the single-pass HBM kernel writes no q_out, mvc_out or mcv_out");
        const size_t need = gather_workspace_bytes(g->m, g->n, p->variant, shots, gather_waves);
        if (ws_bytes < need)
            return fail(BP4_EWORKSPACE, "decode: single-pass HBM workspace %zu < %zu bytes", ws_bytes, need);
        hipError_t e = launch_decode_gather(g->view(dev_graph), g->gather_view(dev_graph), *p, (int32_t)shots,
                                           prior_llr, synd, est, conv, iters, ws, gather_waves, g->with_y,
                                           static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "decode: single-pass HBM launch");
        return BP4_OK;
    }
    if (kernel == BP4_KERNEL_SOA) {
        if (lds_knobs) return fail(BP4_EINVAL, "decode: group_lanes, block_shots and lds_bytes apply to the LDS kernel");
        const size_t need = soa_workspace_bytes(g->m, g->n, g->nnz, p->variant, shots, soa_lanes);
        if (ws_bytes < need) return fail(BP4_EWORKSPACE, "decode: SOA workspace %zu < %zu bytes", ws_bytes, need);
        hipError_t e = launch_decode_soa(g->view(dev_graph), *p, (int32_t)shots, prior_llr, synd, est, conv, iters,
                                         q_out, mvc_out, mcv_out, ws, soa_lanes, soa_block, g->with_y,
                                         static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "decode: SOA launch");
        return BP4_OK;
    }
    size_t max_lds = 0;
    rc = device_max_lds(&max_lds);
    if (rc) return rc;
    LdsLayout L;
    if (p->serial) {
        int G = 0;
        rc = choose_serial_lanes(g, p, requested, requested_S, max_lds, &G);
        if (rc) return rc;
        L = serial_layout(g, p->variant, G);
    } else {
        LaneChoice lc;
        rc = choose_lanes(g, p, requested, requested_S, max_lds, &lc, shots);
        if (rc) return rc;
        L = decode_lds_layout(g->m, g->n, g->nnz, p->variant, lc.group_lanes, lc.block_shots, g->wide());
    }
    MixedArgs args;
    std::memset(&args, 0, sizeof args);
    args.ncodes = 1;
    fill_decode_args(args.codes[0], g, dev_graph, p, shots, prior_llr, synd, est, conv, iters, L,
                     static_cast<unsigned int *>(ws));
    args.codes[0].q_out = q_out;
    args.codes[0].mvc_out = mvc_out;
    args.codes[0].mcv_out = mcv_out;
    args.codes[0].serial = p->serial;
    // the verification outputs map message slots through the graph's slot order
    if (q_out || mvc_out) args.codes[0].css22 = 0;
    if ((size_t)lds_floor > max_lds) return fail(BP4_EINVAL, "decode: lds_bytes %d above the device limit", lds_floor);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_zero_u32(args.codes[0].counter, 1, s);
    if (e != hipSuccess) return hip_fail(e, "decode: zero counter");
    const size_t lds = L.bytes > (size_t)lds_floor ? L.bytes : (size_t)lds_floor;
    e = launch_decode_lds(args, lds, s, nullptr);
    if (e != hipSuccess) return hip_fail(e, "decode: launch");
    return BP4_OK;
}

}  // namespace

extern "C" {

int bp4_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "workspace_bytes: NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0) return fail(BP4_EINVAL, "workspace_bytes: negative shots");
    int k = p->serial ? serial_auto_kernel(g, p->variant) : auto_kernel(g, p->variant);
    if (k == BP4_KERNEL_SOA) k = large_kernel(g, p->variant, p->serial, false);
    *bytes = k == BP4_KERNEL_SOA      ? soa_workspace_bytes(g->m, g->n, g->nnz, p->variant, shots, 0)
             : k == BP4_KERNEL_GATHER ? gather_workspace_bytes(g->m, g->n, p->variant, shots, 0)
                                      : kSmallWorkspace;
    return BP4_OK;
}

int bp4_gather_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, int32_t gather_waves,
                               size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "gather_workspace_bytes: NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0) return fail(BP4_EINVAL, "gather_workspace_bytes: negative shots");
    if (gather_waves != 0 && gather_waves != 4 && gather_waves != 8 && gather_waves != 16)
        return fail(BP4_EINVAL, "gather_workspace_bytes: gather_waves %d not 0, 4, 8 or 16", gather_waves);
    *bytes = gather_workspace_bytes(g->m, g->n, p->variant, shots, gather_waves);
    return BP4_OK;
}

int bp4_soa_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, int32_t soa_lanes,
                            size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "soa_workspace_bytes: NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0 || soa_lanes < 0) return fail(BP4_EINVAL, "soa_workspace_bytes: negative shots or lanes");
    *bytes = soa_workspace_bytes(g->m, g->n, g->nnz, p->variant, shots, soa_lanes);
    return BP4_OK;
}

int bp4_decode(const bp4_graph *g, const void *dev_graph, const bp4_params *p, int64_t shots,
               const float *prior_llr, const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters,
               void *ws, size_t ws_bytes, void *stream)
{
    return decode_common(g, dev_graph, p, nullptr, shots, prior_llr, synd, est, conv, iters, nullptr,
                         nullptr, nullptr, ws, ws_bytes, stream);
}

int bp4_decode_ex(const bp4_graph *g, const void *dev_graph, const bp4_params *p, const bp4_tuning *tune,
                  int64_t shots, const float *prior_llr, const uint8_t *synd, uint8_t *est, uint8_t *conv,
                  int32_t *iters, float *q_out, float *mvc_out, float *mcv_out, void *ws, size_t ws_bytes,
                  void *stream)
{
    return decode_common(g, dev_graph, p, tune, shots, prior_llr, synd, est, conv, iters, q_out, mvc_out,
                         mcv_out, ws, ws_bytes, stream);
}

int bp4_sample(const bp4_graph *g, const void *dev_graph, int64_t shots, int64_t shot0,
               const uint32_t thr[3], uint64_t seed, uint64_t stream_id, uint8_t *err, uint8_t *synd,
               void *stream)
{
    if (!g || !dev_graph || !thr) return fail(BP4_EINVAL, "sample: NULL argument");
    if (shots < 0 || shots > 0x7FFFFFFF || shot0 < 0) return fail(BP4_EINVAL, "sample: shots out of range");
    if ((uint64_t)thr[0] + thr[1] + thr[2] > 0xFFFFFFFFull)
        return fail(BP4_EINVAL, "sample: thresholds sum to 2^32 or more");
    if (shots == 0) return BP4_OK;
    if (!err || !synd) return fail(BP4_EINVAL, "sample: NULL output");
    hipError_t e = launch_sample(g->view(dev_graph), (int32_t)shots, shot0, thr, seed, stream_id, err, synd,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "sample: launch");
    return BP4_OK;
}

int bp4_bookkeep(const bp4_graph *g, const void *dev_graph, int64_t shots, const uint8_t *err,
                 const uint8_t *est, uint8_t *fail_out, int64_t *counts, void *stream)
{
    if (!g || !dev_graph) return fail(BP4_EINVAL, "bookkeep: NULL argument");
    if (g->nlog <= 0) return fail(BP4_EINVAL, "bookkeep: no logical operators set");
    if (shots < 0 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "bookkeep: shots out of range");
    if (shots == 0) return BP4_OK;
    if (!err || !est || !fail_out || !counts) return fail(BP4_EINVAL, "bookkeep: NULL buffer");
    hipError_t e = launch_bookkeep(g->view(dev_graph), (int32_t)shots, err, est, fail_out, counts,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "bookkeep: launch");
    return BP4_OK;
}

}  // extern "C"

extern "C" {

int bp4_mixed_workspace_bytes(int32_t ncodes, size_t *bytes)
{
    if (!bytes) return fail(BP4_EINVAL, "mixed_workspace_bytes: NULL");
    if (ncodes < 1 || ncodes > BP4_MAX_MIXED_CODES)
        return fail(BP4_EINVAL, "mixed_workspace_bytes: ncodes %d outside [1, %d]", ncodes, BP4_MAX_MIXED_CODES);
    *bytes = 256;
    return BP4_OK;
}

int bp4_decode_mixed(int32_t ncodes, const bp4_code_batch *codes, void *ws, size_t ws_bytes, void *stream)
{
    if (!codes || !ws) return fail(BP4_EINVAL, "decode_mixed: NULL argument");
    if (ncodes < 1 || ncodes > BP4_MAX_MIXED_CODES)
        return fail(BP4_EINVAL, "decode_mixed: ncodes %d outside [1, %d]", ncodes, BP4_MAX_MIXED_CODES);
    if (ws_bytes < 256) return fail(BP4_EWORKSPACE, "decode_mixed: workspace %zu < 256 bytes", ws_bytes);
    return bp4::decode_mixed_with(ncodes, codes, static_cast<unsigned int *>(ws), stream);
}

}  // extern "C"

// The mixed launch with its per-code shot-queue heads at `counters` (ncodes words,
// cleared here by a fill kernel before the launch).
int bp4::decode_mixed_with(int32_t ncodes, const bp4_code_batch *codes, unsigned int *counters, void *stream)
{
    if (!codes || !counters) return fail(BP4_EINVAL, "decode_mixed: NULL argument");
    if (ncodes < 1 || ncodes > BP4_MAX_MIXED_CODES)
        return fail(BP4_EINVAL, "decode_mixed: ncodes %d outside [1, %d]", ncodes, BP4_MAX_MIXED_CODES);
    for (int i = 0; i < ncodes; ++i) {
        const bp4_code_batch &c = codes[i];
        if (!c.graph || !c.dev_graph) return fail(BP4_EINVAL, "decode_mixed: code %d has a NULL graph", i);
        int rc = check_params(&c.params);
        if (rc) return rc;
        if (c.shots < 0 || c.shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "decode_mixed: code %d shots out of range", i);
        if (!c.prior_llr) return fail(BP4_EINVAL, "decode_mixed: code %d has a NULL prior", i);
        if (c.shots > 0 && (!c.synd || !c.est || !c.conv || !c.iters))
            return fail(BP4_EINVAL, "decode_mixed: code %d has a NULL buffer", i);
        int rcl = check_lanes(c.group_lanes, c.block_shots, "decode_mixed");
        if (rcl) return rcl;
        if (c.group_lanes == 0 && c.block_shots == 0 && auto_kernel(c.graph, c.params.variant) == BP4_KERNEL_SOA)
            return fail(BP4_EUNSUPPORTED, "decode_mixed: code %d needs the large-code (SOA) kernel", i);
        if (c.params.serial) return fail(BP4_EUNSUPPORTED, "decode_mixed: code %d asks for the serial schedule", i);
    }
    size_t max_lds = 0;
    int rc = device_max_lds(&max_lds);
    if (rc) return rc;
    // largest codes first: their tail is the longest
    std::vector<int> order;
    for (int i = 0; i < ncodes; ++i)
        if (codes[i].shots > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return codes[x].graph->nnz > codes[y].graph->nnz;
    });
    if (order.empty()) return BP4_OK;
    MixedArgs args;
    std::memset(&args, 0, sizeof args);
    args.ncodes = (int32_t)order.size();
    size_t lds = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        const bp4_code_batch &c = codes[order[k]];
        LaneChoice lc;
        rc = choose_lanes(c.graph, &c.params, c.group_lanes, c.block_shots, max_lds, &lc, c.shots);
        if (rc) return rc;
        const LdsLayout L = decode_lds_layout(c.graph->m, c.graph->n, c.graph->nnz, c.params.variant, lc.group_lanes,
                                              lc.block_shots, c.graph->wide());
        lds = L.bytes > lds ? L.bytes : lds;
        fill_decode_args(args.codes[k], c.graph, c.dev_graph, &c.params, c.shots, c.prior_llr, c.synd, c.est,
                         c.conv, c.iters, L, counters + k);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_zero_u32(counters, args.ncodes, s);
    if (e != hipSuccess) return hip_fail(e, "decode_mixed: zero counters");
    e = launch_decode_lds(args, lds, s, nullptr);
    if (e != hipSuccess) return hip_fail(e, "decode_mixed: launch");
    return BP4_OK;
}

int bp4::report_error(int code, const char *what, hipError_t e)
{
    return e == hipSuccess ? fail(code, "%s", what) : hip_fail(e, what);
}

extern "C" {

int bp4_plain_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "plain_workspace_bytes: NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "plain_workspace_bytes: shots out of range");
    *bytes = plain_workspace_bytes(g->n, g->nnz, p->variant, shots);
    return BP4_OK;
}

int bp4_decode_plain(const bp4_graph *g, const void *dev_graph, const bp4_params *p, int64_t shots,
                     const float *prior_llr, const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters,
                     void *ws, size_t ws_bytes, void *stream, int32_t *iterations_run)
{
    if (!g || !dev_graph) return fail(BP4_EINVAL, "decode_plain: NULL graph");
    int rc = check_params(p);
    if (rc) return rc;
    if (shots < 0 || shots > 0x7FFFFFFF) return fail(BP4_EINVAL, "decode_plain: shots out of range");
    if (!prior_llr) return fail(BP4_EINVAL, "decode_plain: NULL prior");
    if (iterations_run) *iterations_run = 0;
    if (p->serial) return fail(BP4_EUNSUPPORTED, "decode_plain: flooding schedule only");
    if (p->variant == BP4_AEWA) return fail(BP4_EUNSUPPORTED, "decode_plain: AEWA restarts need the persistent kernels");
    if (shots == 0) return BP4_OK;
    if (!synd || !est || !conv || !iters || !ws) return fail(BP4_EINVAL, "decode_plain: NULL buffer");
    const size_t need = plain_workspace_bytes(g->n, g->nnz, p->variant, shots);
    if (ws_bytes < need) return fail(BP4_EWORKSPACE, "decode_plain: workspace %zu < %zu bytes", ws_bytes, need);
    int32_t it = 0;
    hipError_t e = run_plain(g->view(dev_graph), *p, (int32_t)shots, prior_llr, synd, est, conv, iters, ws,
                             static_cast<hipStream_t>(stream), &it);
    if (e != hipSuccess) return hip_fail(e, "decode_plain");
    if (iterations_run) *iterations_run = it;
    return BP4_OK;
}

}  // extern "C"

extern "C" int bp4_lds_layout_bytes(const bp4_graph *g, const bp4_params *p, int32_t group_lanes,
                                    int32_t block_shots, size_t *bytes)
{
    if (!g || !bytes) return fail(BP4_EINVAL, "lds_layout_bytes: NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    int G = group_lanes, S = block_shots;
    if (p->serial) {
        if (S != 0 || (G != 1 && G != 2 && G != 4 && G != 8 && G != 16 && G != 32 && G != 64))
            return fail(BP4_EINVAL, "lds_layout_bytes: the serial schedule takes group_lanes 1 ... 64 and no block_shots");
        *bytes = serial_layout(g, p->variant, G).bytes;
        return BP4_OK;
    }
    rc = check_lanes(G, S, "lds_layout_bytes");
    if (rc) return rc;
    if (G == 0 && S == 0) return fail(BP4_EINVAL, "lds_layout_bytes: no lane mapping given");
    if (G > 64 || S > 0) {
        if (S == 0) S = kLdsBlock / G;
        G = kLdsBlock;
    }
    if (!decode_lds_fits(g->m, g->n, G, S)) return fail(BP4_EINVAL, "lds_layout_bytes: more than 64 checks per lane");
    *bytes = decode_lds_layout(g->m, g->n, g->nnz, p->variant, G, S, g->wide()).bytes;
    return BP4_OK;
}
