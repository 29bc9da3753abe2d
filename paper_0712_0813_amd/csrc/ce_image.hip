// Grid images: the whole state of one simulation as a flat host buffer, and a
// resumed run from it (the paper's resumable grid image, "Overview" section).
// The layout is documented with ce_image_header in ce.h.
#include <string.h>

#include "ce_sim.hpp"

using namespace ce;
using namespace ce::host;

static_assert(sizeof(ce_image_header) == 512, "image header must stay 512 bytes");

namespace {

constexpr size_t kHeader = sizeof(ce_image_header);

size_t storage_elem(const ce_params &p) { return p.precision == CE_FP64 ? 8 : 4; }

size_t array_bytes(const ce_params &p) { return (size_t)sites_of(&p) * storage_elem(p); }

size_t image_total(const ce_params &p)
{
    return kHeader + sizeof(Scalars) + (size_t)kLogCap * sizeof(ce_energy) + 2 * (size_t)p.nfields * array_bytes(p);
}

bool same_double(double a, double b) { return memcmp(&a, &b, sizeof(double)) == 0; }

// Physics parameters equal bit for bit (stream and arena excluded).
const char *param_mismatch(const ce_params &a, const ce_params &b)
{
    if (a.dims != b.dims) return "dims";
    if (a.N != b.N) return "N";
    if (a.nfields != b.nfields) return "nfields";
    if (a.precision != b.precision) return "precision";
    if (a.model != b.model) return "model";
    if (a.expansion != b.expansion) return "expansion";
    if (!same_double(a.L, b.L)) return "L";
    if (!same_double(a.dt, b.dt)) return "dt";
    if (!same_double(a.lambda, b.lambda)) return "lambda";
    for (int i = 0; i < CE_MAX_FIELDS; i++) {
        if (!same_double(a.G[i], b.G[i])) return "G";
        if (!same_double(a.mu2[i], b.mu2[i])) return "mu2";
    }
    if (!same_double(a.kappa, b.kappa)) return "kappa";
    if (!same_double(a.vacuum, b.vacuum)) return "vacuum";
    if (a.nterms != b.nterms) return "nterms";
    for (int t = 0; t < a.nterms && t < CE_MAX_TERMS; t++) {
        if (!same_double(a.terms[t].coef, b.terms[t].coef)) return "terms (coefficient)";
        for (int i = 0; i < CE_MAX_FIELDS; i++)
            if (a.terms[t].exp[i] != b.terms[t].exp[i]) return "terms (exponent)";
    }
    return nullptr;
}

// Header checks shared by ce_image_params and ce_restore_image.
ce_status parse_header(const void *buf, size_t bytes, ce_image_header *h, ce_params *p)
{
    if (!buf) return fail(CE_EINVAL, "image buffer is NULL");
    if (bytes < kHeader) return fail(CE_EINVAL, "image of %zu bytes is shorter than its header", bytes);
    memcpy(h, buf, kHeader);
    if (memcmp(h->magic, CE_IMAGE_MAGIC, 8) != 0) return fail(CE_EINVAL, "not a grid image (bad magic)");
    if (h->version != CE_IMAGE_VERSION) return fail(CE_EINVAL, "grid image version %u, expected %u", h->version,
                                                    CE_IMAGE_VERSION);
    if (h->header_bytes != kHeader) return fail(CE_EINVAL, "grid image header of %u bytes", h->header_bytes);
    memset(p, 0, sizeof(*p));
    p->dims = h->dims;
    p->N = h->N;
    p->nfields = h->nfields;
    p->precision = h->precision;
    p->model = h->model;
    p->expansion = h->expansion;
    p->L = h->L;
    p->dt = h->dt;
    p->lambda = h->lambda;
    for (int i = 0; i < CE_MAX_FIELDS; i++) {
        p->G[i] = h->G[i];
        p->mu2[i] = h->mu2[i];
    }
    p->kappa = h->kappa;
    p->vacuum = h->vacuum;
    p->nterms = h->nterms;
    if (p->nterms < 0 || p->nterms > CE_MAX_TERMS) return fail(CE_EINVAL, "grid image holds %d model terms", p->nterms);
    for (int t = 0; t < p->nterms; t++) p->terms[t] = h->terms[t];
    ce_status st = validate(p);
    if (st != CE_OK) return st;
    if (h->field_bytes != array_bytes(*p)) return fail(CE_EINVAL, "grid image field size does not match N");
    if (h->state_bytes > (1u << 20) || h->ring_bytes > (1u << 30) ||
        h->total_bytes != kHeader + h->state_bytes + h->ring_bytes + 2 * (uint64_t)p->nfields * h->field_bytes)
        return fail(CE_EINVAL, "grid image section sizes are inconsistent");
    if (bytes < h->total_bytes)
        return fail(CE_EINVAL, "grid image truncated: %zu of %llu bytes", bytes, (unsigned long long)h->total_bytes);
    return CE_OK;
}

}  // namespace

extern "C" {

ce_status ce_image_bytes(const ce_sim *s, size_t *out)
{
    if (!s || !out) return fail(CE_EINVAL, "NULL argument");
    *out = image_total(s->p);
    return CE_OK;
}

ce_status ce_save_image(ce_sim *s, void *buf, size_t bytes)
{
    if (!s || !buf) return fail(CE_EINVAL, "NULL argument");
    if (!s->started) return fail(CE_ESTATE, "no grid image before every field is loaded");
    const ce_params &p = s->p;
    const size_t total = image_total(p);
    if (bytes < total) return fail(CE_EINVAL, "image buffer holds %zu bytes, %zu needed", bytes, total);
    CE_HIP(hipStreamSynchronize(s->stream));

    ce_image_header h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, CE_IMAGE_MAGIC, 8);
    h.version = CE_IMAGE_VERSION;
    h.header_bytes = (uint32_t)kHeader;
    h.dims = p.dims;
    h.N = p.N;
    h.nfields = p.nfields;
    h.precision = p.precision;
    h.model = p.model;
    h.expansion = p.expansion;
    h.L = p.L;
    h.dt = p.dt;
    h.lambda = p.lambda;
    for (int i = 0; i < CE_MAX_FIELDS; i++) {
        h.G[i] = p.G[i];
        h.mu2[i] = p.mu2[i];
    }
    h.kappa = p.kappa;
    h.vacuum = p.vacuum;
    h.nterms = p.nterms;
    for (int t = 0; t < p.nterms; t++) h.terms[t] = p.terms[t];
    h.step = s->step;
    h.launch = s->launch;
    h.launch.grid = s->lat.nblocks;
    h.state_bytes = sizeof(Scalars);
    h.ring_bytes = (uint64_t)kLogCap * sizeof(ce_energy);
    h.field_bytes = array_bytes(p);
    h.total_bytes = total;

    char *out = static_cast<char *>(buf);
    memcpy(out, &h, kHeader);
    size_t off = kHeader;
    CE_HIP(hipMemcpyAsync(out + off, s->lat.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s->stream));
    off += sizeof(Scalars);
    CE_HIP(hipMemcpyAsync(out + off, s->lat.ring, h.ring_bytes, hipMemcpyDeviceToHost, s->stream));
    off += h.ring_bytes;
    for (int i = 0; i < p.nfields; i++) {
        CE_HIP(hipMemcpyAsync(out + off, s->lat.d[s->cur][i], h.field_bytes, hipMemcpyDeviceToHost, s->stream));
        off += h.field_bytes;
        CE_HIP(hipMemcpyAsync(out + off, s->lat.p[s->cur][i], h.field_bytes, hipMemcpyDeviceToHost, s->stream));
        off += h.field_bytes;
    }
    CE_HIP(hipStreamSynchronize(s->stream));
    return CE_OK;
}

ce_status ce_image_params(const void *buf, size_t bytes, ce_params *out)
{
    if (!out) return fail(CE_EINVAL, "out is NULL");
    ce_image_header h;
    ce_params p;
    ce_status st = parse_header(buf, bytes, &h, &p);
    if (st != CE_OK) return st;
    *out = p;
    return CE_OK;
}

ce_status ce_restore_image(ce_sim *s, const void *buf, size_t bytes)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    ce_image_header h;
    ce_params p;
    ce_status st = parse_header(buf, bytes, &h, &p);
    if (st != CE_OK) return st;
    if (h.state_bytes != sizeof(Scalars) || h.ring_bytes != (uint64_t)kLogCap * sizeof(ce_energy))
        return fail(CE_EINVAL, "grid image written by a build with another state layout");
    if (const char *what = param_mismatch(p, s->p))
        return fail(CE_EINVAL, "grid image parameter %s differs from the simulation's", what);
    if (h.step < 0) return fail(CE_EINVAL, "grid image step is negative");
    const char *in = static_cast<const char *>(buf);
    Scalars sc;
    memcpy(&sc, in + kHeader, sizeof(sc));
    if (sc.step != h.step) return fail(CE_EINVAL, "grid image scalar state is at another step than its header");

    // the launch first: it is the only step that can fail without touching
    // the device state
    const ce_launch old = s->launch;
    const Lattice saved = s->lat;
    st = apply_launch(s, h.launch);
    if (st != CE_OK) {
        s->launch = old;
        s->lat = saved;
        return st;
    }
    CE_HIP(hipStreamSynchronize(s->stream));
    size_t off = kHeader;
    CE_HIP(hipMemcpyAsync(s->lat.sc, in + off, sizeof(Scalars), hipMemcpyHostToDevice, s->stream));
    off += sizeof(Scalars);
    CE_HIP(hipMemcpyAsync(s->lat.ring, in + off, h.ring_bytes, hipMemcpyHostToDevice, s->stream));
    off += h.ring_bytes;
    for (int i = 0; i < p.nfields; i++) {
        CE_HIP(hipMemcpyAsync(s->lat.d[0][i], in + off, h.field_bytes, hipMemcpyHostToDevice, s->stream));
        off += h.field_bytes;
        CE_HIP(hipMemcpyAsync(s->lat.p[0][i], in + off, h.field_bytes, hipMemcpyHostToDevice, s->stream));
        off += h.field_bytes;
    }
    CE_HIP(hipStreamSynchronize(s->stream));
    for (int i = 0; i < CE_MAX_FIELDS; i++) s->m_host[i] = sc.m[i];
    s->cur = 0;
    s->step = h.step;
    s->loaded = (1u << p.nfields) - 1;
    s->started = true;
    return CE_OK;
}

}  // extern "C"
