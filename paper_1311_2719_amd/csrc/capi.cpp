// The C ABI of libstagcg (declared in include/stagcg.h): argument checking and
// dispatch into the runtime.  No exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "runtime.hpp"
#include "serve.hpp"

namespace stag {
const char *last_error_cstr();
int validate_cg_params(const stag_cg_params &p);
}  // namespace stag

using namespace stag;

#define STAG_GUARD_BEGIN try {
#define STAG_GUARD_END                                                              \
    }                                                                               \
    catch (const std::bad_alloc &) { return set_error(STAG_ENOMEM, "host allocation failed"); } \
    catch (...) { return set_error(STAG_EHIP, "internal error"); }

static hipStream_t pick_stream(stag_ctx *ctx, void *stream)
{
    return stream ? (hipStream_t)stream : reinterpret_cast<Ctx *>(ctx)->stream;
}

static bool dims_ok(const int32_t *d)
{
    if (!d)
        return false;
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        if (d[i] < 2 || (d[i] & 1))
            return false;
        v *= d[i];
    }
    // checkerboard indices are 32-bit: V/2 must fit
    return v / 2 < (int64_t)1 << 31 && (v / 2) * 8 * 9 < ((int64_t)1 << 62);
}

extern "C" {

const char *stag_version(void) { return "stagcg 1.0 (gfx950)"; }

const char *stag_last_error(const stag_ctx *) { return last_error_cstr(); }

int stag_create(int device, void *arena_dev, size_t arena_bytes, void *stream, stag_ctx **out)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!out || !arena_dev)
        return set_error(STAG_EINVAL, "stag_create: NULL arena or output pointer");
    if (arena_bytes < ((size_t)1 << 20))
        return set_error(STAG_EINVAL, "stag_create: arena must be at least 1 MiB");
    int ndev = 0;
    STAG_HIP_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return set_error(STAG_EINVAL, "stag_create: device %d out of range (%d devices)", device, ndev);
    DeviceGuard dg(device);
    // the fixed workspace of stag_cg_solve_noalloc: its address on this device
    int rc = noalloc_setup(device);
    if (rc != STAG_OK)
        return rc;
    Ctx *c = new Ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->arena.init(arena_dev, arena_bytes);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    *out = reinterpret_cast<stag_ctx *>(c);
    return STAG_OK;
    STAG_GUARD_END
}

int stag_destroy(stag_ctx *ctx)
{
    STAG_GUARD_BEGIN
    if (!ctx)
        return set_error(STAG_EINVAL, "stag_destroy: NULL context");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    c->server.reset();
    drop_cached_batches(c, -1);
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->fields.clear();
    }
    delete c;
    return STAG_OK;
    STAG_GUARD_END
}

int stag_arena_usage(const stag_ctx *ctx, size_t *used, size_t *total)
{
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
    if (used)
        *used = c->arena.used();
    if (total)
        *total = c->arena.total();
    return STAG_OK;
}

int stag_set_gauge(stag_ctx *ctx, const int32_t dims[4], const double *links, int32_t links_on_device,
                   int32_t t_antiperiodic, int32_t *gauge_id)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !links || !gauge_id)
        return set_error(STAG_EINVAL, "stag_set_gauge: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_set_gauge: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    auto f = std::make_shared<GaugeField>();
    memcpy(f->dims, dims, sizeof(f->dims));
    f->tap = t_antiperiodic ? 1 : 0;
    f->g = make_geom(dims);
    f->g.tap = f->tap;
    const size_t Vh = f->g.Vh;
    hipStream_t s = c->stream;
    // the caller's links on the device (staged through the arena if on the host)
    const size_t in_bytes = 2 * Vh * 4 * 9 * 16;
    const double *src = links;
    void *staging = nullptr;
    if (!links_on_device) {
        staging = c->arena.alloc(in_bytes);
        if (!staging)
            return set_error(STAG_ENOMEM, "stag_set_gauge: arena exhausted (staging %zu bytes)", in_bytes);
        hipError_t e = hipMemcpyAsync(staging, links, in_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            c->arena.release(staging);
            return set_error(STAG_EHIP, "stag_set_gauge: copy failed: %s", hipGetErrorString(e));
        }
        src = (const double *)staging;
    }
    struct StagingGuard {
        Arena &arena;
        void *p;
        ~StagingGuard() { arena.release(p); }
    } staging_guard{c->arena, staging};
    // two stored rows when every folded link admits it (STAG_LINK_ROWS=3 keeps all three)
    bool two_rows = false;
    int rc = gauge_check(c, f->g, src, s, two_rows);
    if (rc != STAG_OK)
        return rc;
    const char *rows_env = getenv("STAG_LINK_ROWS");
    f->rows = two_rows && !(rows_env && atoi(rows_env) == 3) ? 2 : 3;
    f->nt_links = nt_links_for(*f);
    for (int p = 0; p < 3; ++p) {
        const size_t lb = (size_t)2 * link_parity_entries(f->rows, (int)Vh) * link_entry_bytes_of(p);
        f->links[p] = c->arena.alloc(lb);
        f->bytes += lb;
    }
    f->nbr = (int32_t *)c->arena.alloc(2 * 8 * Vh * sizeof(int32_t));
    f->bytes += 2 * 8 * Vh * sizeof(int32_t);
    auto release_all = [&]() {
        for (int p = 0; p < 3; ++p)
            c->arena.release(f->links[p]);
        c->arena.release(f->nbr);
    };
    if (!f->links[0] || !f->links[1] || !f->links[2] || !f->nbr) {
        release_all();
        return set_error(STAG_ENOMEM, "stag_set_gauge: arena exhausted (%zu bytes needed)", f->bytes);
    }
    rc = gauge_prepare(f.get(), src, s);
    if (rc != STAG_OK) {
        release_all();
        return rc;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    f->id = c->next_id++;
    c->fields[f->id] = f;
    *gauge_id = f->id;
    return STAG_OK;
    STAG_GUARD_END
}

int stag_free_gauge(stag_ctx *ctx, int32_t gauge_id)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    std::shared_ptr<GaugeField> f;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->fields.find(gauge_id);
        if (it == c->fields.end())
            return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
        if (it->second->users.load() > 0)
            return set_error(STAG_EBUSY, "gauge field %d has %d pending requests", gauge_id,
                             it->second->users.load());
        f = it->second;
        c->fields.erase(it);
    }
    if (c->server)
        c->server->drop_field(gauge_id);
    drop_cached_batches(c, gauge_id);
    (void)hipDeviceSynchronize();
    for (int p = 0; p < 3; ++p)
        c->arena.release(f->links[p]);
    c->arena.release(f->nbr);
    return STAG_OK;
    STAG_GUARD_END
}

int stag_gauge_dims(stag_ctx *ctx, int32_t gauge_id, int32_t dims[4])
{
    if (!ctx || !dims)
        return set_error(STAG_EINVAL, "NULL argument");
    auto f = reinterpret_cast<Ctx *>(ctx)->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    memcpy(dims, f->dims, sizeof(f->dims));
    return STAG_OK;
}

int stag_gauge_link_rows(stag_ctx *ctx, int32_t gauge_id, int32_t *rows)
{
    if (!ctx || !rows)
        return set_error(STAG_EINVAL, "NULL argument");
    auto f = reinterpret_cast<Ctx *>(ctx)->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    *rows = f->rows;
    return STAG_OK;
}

// ---- Wilson fermions -----------------------------------------------------------------

int stag_set_gauge_wilson(stag_ctx *ctx, const int32_t dims[4], const double *links, int32_t links_on_device,
                          int32_t t_antiperiodic, int32_t *gauge_id)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !links || !gauge_id)
        return set_error(STAG_EINVAL, "stag_set_gauge_wilson: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_set_gauge_wilson: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    auto f = std::make_shared<GaugeField>();
    f->kind = FIELD_WILSON;
    memcpy(f->dims, dims, sizeof(f->dims));
    f->tap = t_antiperiodic ? 1 : 0;
    f->g = make_geom(dims);
    f->g.tap = f->tap;
    const size_t Vh = f->g.Vh;
    hipStream_t s = c->stream;
    const size_t in_bytes = 2 * Vh * 4 * 9 * 16;
    const double *src = links;
    void *staging = nullptr;
    if (!links_on_device) {
        staging = c->arena.alloc(in_bytes);
        if (!staging)
            return set_error(STAG_ENOMEM, "stag_set_gauge_wilson: arena exhausted (staging %zu bytes)", in_bytes);
        hipError_t e = hipMemcpyAsync(staging, links, in_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            c->arena.release(staging);
            return set_error(STAG_EHIP, "stag_set_gauge_wilson: copy failed: %s", hipGetErrorString(e));
        }
        src = (const double *)staging;
    }
    const int rc = wilson_prepare(c, f.get(), src, s);
    c->arena.release(staging);
    if (rc != STAG_OK)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    f->id = c->next_id++;
    c->fields[f->id] = f;
    *gauge_id = f->id;
    return STAG_OK;
    STAG_GUARD_END
}

int stag_pack_spinor(stag_ctx *ctx, const int32_t dims[4], const double *lex, double *eo, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !lex || !eo)
        return set_error(STAG_EINVAL, "stag_pack_spinor: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_pack_spinor: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return launch_pack_spinor(make_geom(dims), lex, eo, 1, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_unpack_spinor(stag_ctx *ctx, const int32_t dims[4], const double *eo, double *lex, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !lex || !eo)
        return set_error(STAG_EINVAL, "stag_unpack_spinor: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_unpack_spinor: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return launch_pack_spinor(make_geom(dims), lex, const_cast<double *>(eo), 0, pick_stream(ctx, stream));
    STAG_GUARD_END
}

static int wilson_field(stag_ctx *ctx, int32_t gauge_id, std::shared_ptr<GaugeField> &f)
{
    f = reinterpret_cast<Ctx *>(ctx)->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_WILSON)
        return set_error(STAG_EINVAL, "gauge id %d holds staggered links", gauge_id);
    return STAG_OK;
}

int stag_wilson_dslash(stag_ctx *ctx, int32_t gauge_id, int32_t out_parity, const double *in, double *out,
                       void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !in || !out)
        return set_error(STAG_EINVAL, "stag_wilson_dslash: NULL argument");
    std::shared_ptr<GaugeField> f;
    int rc = wilson_field(ctx, gauge_id, f);
    if (rc != STAG_OK)
        return rc;
    if (out_parity < STAG_EVEN || out_parity > STAG_ALL)
        return set_error(STAG_EINVAL, "stag_wilson_dslash: bad parity %d", out_parity);
    const char *a0 = (const char *)in, *b0 = (const char *)out;
    const size_t fb = (size_t)2 * 12 * f->g.Vh * 16;
    if (a0 < b0 + fb && b0 < a0 + fb)
        return set_error(STAG_EINVAL, "stag_wilson_dslash: in and out must not overlap");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return wilson_dslash(c, f.get(), out_parity, in, out, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_wilson_solve(stag_ctx *ctx, int32_t gauge_id, double kappa, double tol, int32_t maxiter, const double *b,
                      double *x, void *stream, stag_cg_info *info)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !b || !x)
        return set_error(STAG_EINVAL, "stag_wilson_solve: NULL argument");
    std::shared_ptr<GaugeField> f;
    int rc = wilson_field(ctx, gauge_id, f);
    if (rc != STAG_OK)
        return rc;
    if (!(kappa > 0 && kappa < INFINITY) || !(tol > 0 && tol < 1) || maxiter < 0)
        return set_error(STAG_EINVAL, "stag_wilson_solve: kappa > 0, 0 < tol < 1 and maxiter >= 0 are required");
    const char *a0 = (const char *)b, *b0 = (const char *)x;
    const size_t fb = (size_t)2 * 12 * f->g.Vh * 16;
    if (a0 < b0 + fb && b0 < a0 + fb)
        return set_error(STAG_EINVAL, "stag_wilson_solve: b and x must not overlap");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return wilson_cg_solve(c, f.get(), kappa, tol, maxiter, b, x, pick_stream(ctx, stream), info);
    STAG_GUARD_END
}

int stag_pack_fermion(stag_ctx *ctx, const int32_t dims[4], const double *lex, double *eo, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !lex || !eo)
        return set_error(STAG_EINVAL, "stag_pack_fermion: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_pack_fermion: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return launch_pack(make_geom(dims), lex, eo, 1, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_unpack_fermion(stag_ctx *ctx, const int32_t dims[4], const double *eo, double *lex, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !lex || !eo)
        return set_error(STAG_EINVAL, "stag_unpack_fermion: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_unpack_fermion: every extent must be even and >= 2");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return launch_pack(make_geom(dims), lex, const_cast<double *>(eo), 0, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_dslash(stag_ctx *ctx, int32_t gauge_id, int32_t out_parity, int64_t offset, int64_t count, const void *in,
                void *out, int32_t accumulate, int32_t precision, int32_t on_device, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !in || !out)
        return set_error(STAG_EINVAL, "stag_dslash: NULL argument");
    if (in == out)
        return set_error(STAG_EINVAL, "stag_dslash: in and out must not overlap");
    if (precision < STAG_F64 || precision > STAG_F16)
        return set_error(STAG_EINVAL, "stag_dslash: unknown precision %d", precision);
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    const int64_t Vh = f->g.Vh;
    if (out_parity < STAG_EVEN || out_parity > STAG_ALL)
        return set_error(STAG_EINVAL, "stag_dslash: bad parity %d", out_parity);
    if (count < 0)
        count = Vh - offset;
    if (out_parity == STAG_ALL && (offset != 0 || count != Vh))
        return set_error(STAG_EINVAL, "stag_dslash: STAG_ALL takes offset 0 and count -1");
    if (offset < 0 || offset > Vh || count < 0 || offset + count > Vh)
        return set_error(STAG_EINVAL, "stag_dslash: range [%lld, %lld) outside [0, %lld)", (long long)offset,
                         (long long)(offset + count), (long long)Vh);
    const size_t hb = (size_t)Vh * spinor_bytes_of(precision);  // bytes of one parity half
    const char *a0 = (const char *)in, *b0 = (const char *)out;
    if (a0 < b0 + 2 * hb && b0 < a0 + 2 * hb)
        return set_error(STAG_EINVAL, "stag_dslash: in and out must not overlap");
    if (count == 0)
        return STAG_OK;
    DeviceGuard dg(c->device);
    hipStream_t s = pick_stream(ctx, stream);
    if (on_device)
        return dslash(c, f.get(), precision, out_parity, offset, count, in, out, accumulate, s);
    // host arrays: stage through the arena (the paper's copyin / copyout)
    struct Staging {
        Arena &arena;
        void *p;
        ~Staging() { arena.release(p); }
    } st{c->arena, c->arena.alloc(4 * hb)};
    if (!st.p)
        return set_error(STAG_ENOMEM, "stag_dslash: arena exhausted (staging %zu bytes)", 4 * hb);
    char *din = (char *)st.p, *dout = din + 2 * hb;
    // the written output range: per parity, one piece per colour plane
    // (FP64 / FP32 [colour][Vh]) or one piece of records (FP16)
    const size_t esz = precision == STAG_F16 ? 16 : spinor_bytes_of(precision) / 3;
    const int planes = precision == STAG_F16 ? 1 : 3;
    auto copy_range = [&](int par, hipMemcpyKind kind) -> hipError_t {
        for (int pl = 0; pl < planes; ++pl) {
            const size_t o = (size_t)par * hb + ((size_t)pl * Vh + offset) * esz;
            hipError_t e = kind == hipMemcpyHostToDevice
                               ? hipMemcpyAsync(dout + o, b0 + o, (size_t)count * esz, kind, s)
                               : hipMemcpyAsync((char *)out + o, dout + o, (size_t)count * esz, kind, s);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    if (out_parity == STAG_ALL)
        STAG_HIP_CHECK(hipMemcpyAsync(din, in, 2 * hb, hipMemcpyHostToDevice, s));
    else
        STAG_HIP_CHECK(hipMemcpyAsync(din + (1 - out_parity) * hb, a0 + (1 - out_parity) * hb, hb,
                                      hipMemcpyHostToDevice, s));
    for (int par = 0; par < 2 && accumulate; ++par)
        if (out_parity == STAG_ALL || out_parity == par)
            STAG_HIP_CHECK(copy_range(par, hipMemcpyHostToDevice));
    int rc = dslash(c, f.get(), precision, out_parity, offset, count, din, dout, accumulate, s);
    if (rc != STAG_OK) {
        (void)hipStreamSynchronize(s);
        return rc;
    }
    for (int par = 0; par < 2; ++par)
        if (out_parity == STAG_ALL || out_parity == par)
            STAG_HIP_CHECK(copy_range(par, hipMemcpyDeviceToHost));
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    return STAG_OK;
    STAG_GUARD_END
}

int stag_convert_fermion(stag_ctx *ctx, const int32_t dims[4], const void *in, int32_t in_precision, void *out,
                         int32_t out_precision, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !in || !out)
        return set_error(STAG_EINVAL, "stag_convert_fermion: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_convert_fermion: every extent must be even and >= 2");
    if (in_precision < STAG_F64 || in_precision > STAG_F16 || out_precision < STAG_F64 || out_precision > STAG_F16)
        return set_error(STAG_EINVAL, "stag_convert_fermion: unknown precision");
    const Geom g = make_geom(dims);
    const char *a0 = (const char *)in, *b0 = (const char *)out;
    const size_t na = (size_t)2 * g.Vh * spinor_bytes_of(in_precision);
    const size_t nb = (size_t)2 * g.Vh * spinor_bytes_of(out_precision);
    if (a0 < b0 + nb && b0 < a0 + na)
        return set_error(STAG_EINVAL, "stag_convert_fermion: in and out must not overlap");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return convert_fermion(g, in_precision, in, out_precision, out, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_cg_solve(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params, const double *b, double *x,
                  double *y, int32_t on_device, void *stream, stag_cg_info *info)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !params || !b || !x)
        return set_error(STAG_EINVAL, "stag_cg_solve: NULL argument");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    int rc = validate_cg_params(*params);
    if (rc != STAG_OK)
        return rc;
    DeviceGuard dg(c->device);
    hipStream_t s = pick_stream(ctx, stream);
    if (on_device) {
        double *ys[1] = {y};
        return cg_solve_batch(c, f, 1, params, &b, &x, ys, s, info);
    }
    // host arrays: b in, x (and y) out, through the arena (the paper's data
    // region: copyin of the source, copyout of the solution)
    const size_t hb = (size_t)f->g.Vh * 48, hd = (size_t)f->g.Vh * 6;  // bytes / doubles per parity half
    const size_t nbuf = y ? 3 : 2;
    struct Staging {
        Arena &arena;
        void *p;
        ~Staging() { arena.release(p); }
    } st{c->arena, c->arena.alloc(nbuf * 2 * hb)};
    if (!st.p)
        return set_error(STAG_ENOMEM, "stag_cg_solve: arena exhausted (staging %zu bytes)", nbuf * 2 * hb);
    double *db = (double *)st.p, *dx = db + 2 * hd, *dy = y ? dx + 2 * hd : nullptr;
    const int par = params->parity;
    auto solved = [&](int p) { return par == STAG_ALL || par == p; };
    for (int p = 0; p < 2; ++p)
        if (solved(p))
            STAG_HIP_CHECK(hipMemcpyAsync(db + p * hd, b + p * hd, hb, hipMemcpyHostToDevice, s));
    const double *bs[1] = {db};
    double *xs[1] = {dx}, *ys[1] = {dy};
    rc = cg_solve_batch(c, f, 1, params, bs, xs, ys, s, info);
    // x holds the last iterate also when the solve ran and did not converge
    const bool ran = rc == STAG_OK || rc == STAG_ENOCONV || rc == STAG_EBREAKDOWN || rc == STAG_ENONFINITE;
    const std::string msg = rc != STAG_OK ? std::string(last_error_cstr()) : std::string();
    for (int p = 0; p < 2 && ran; ++p) {
        if (solved(p))
            STAG_HIP_CHECK(hipMemcpyAsync(x + p * hd, dx + p * hd, hb, hipMemcpyDeviceToHost, s));
        if (y && solved(1 - p))
            STAG_HIP_CHECK(hipMemcpyAsync(y + p * hd, dy + p * hd, hb, hipMemcpyDeviceToHost, s));
    }
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    if (rc != STAG_OK)
        return set_error(rc, "%s", msg.c_str());
    return STAG_OK;
    STAG_GUARD_END
}

int stag_fermion_force(stag_ctx *ctx, int32_t gauge_id, const double *w, double *force, double coeff,
                       int32_t accumulate, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !w || !force)
        return set_error(STAG_EINVAL, "stag_fermion_force: NULL argument");
    if (!std::isfinite(coeff))
        return set_error(STAG_EINVAL, "stag_fermion_force: coefficient must be finite");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    const size_t wb = (size_t)2 * 3 * f->g.Vh * 16, fb = (size_t)2 * f->g.Vh * 4 * 9 * 16;
    const char *a0 = (const char *)w, *b0 = (const char *)force;
    if (a0 < b0 + fb && b0 < a0 + wb)
        return set_error(STAG_EINVAL, "stag_fermion_force: w and force must not overlap");
    DeviceGuard dg(c->device);
    return fermion_force(f.get(), w, force, coeff, accumulate, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_gauge_force(stag_ctx *ctx, const int32_t dims[4], const double *links, double beta, double *force,
                     double coeff, int32_t accumulate, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !links || !force)
        return set_error(STAG_EINVAL, "stag_gauge_force: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_gauge_force: every extent must be even and >= 2");
    if (!std::isfinite(beta) || !std::isfinite(coeff))
        return set_error(STAG_EINVAL, "stag_gauge_force: beta and coeff must be finite");
    const size_t n = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * 4 * 9 * 16;
    const char *a0 = (const char *)links, *b0 = (const char *)force;
    if (a0 < b0 + n && b0 < a0 + n)
        return set_error(STAG_EINVAL, "stag_gauge_force: links and force must not overlap");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return gauge_force(dims, links, force, beta, coeff, accumulate, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_pseudofermion(stag_ctx *ctx, int32_t gauge_id, const double *chi, double *phi, double mass, void *stream)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !chi || !phi)
        return set_error(STAG_EINVAL, "stag_pseudofermion: NULL argument");
    if (!std::isfinite(mass))
        return set_error(STAG_EINVAL, "stag_pseudofermion: mass must be finite");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    const size_t n = (size_t)2 * 3 * f->g.Vh * 16;
    const char *a0 = (const char *)chi, *b0 = (const char *)phi;
    if (a0 < b0 + n && b0 < a0 + n)
        return set_error(STAG_EINVAL, "stag_pseudofermion: chi and phi must not overlap");
    DeviceGuard dg(c->device);
    return pseudofermion(c, f.get(), chi, phi, mass, pick_stream(ctx, stream));
    STAG_GUARD_END
}

int stag_md_trajectory(stag_ctx *ctx, const int32_t dims[4], double *links, double *momenta, const double *phi,
                       const stag_md_params *params, void *stream, stag_md_info *info)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !links || !momenta || !phi || !params)
        return set_error(STAG_EINVAL, "stag_md_trajectory: NULL argument");
    if (!dims_ok(dims))
        return set_error(STAG_EINVAL, "stag_md_trajectory: every extent must be even and >= 2");
    const stag_md_params &p = *params;
    if (!(p.mass > 0) || !std::isfinite(p.mass) || !(p.eps > 0) || !std::isfinite(p.eps) || !std::isfinite(p.beta) ||
        !(p.tol > 0) || p.nsteps < 1 || p.maxiter < 1 || p.precision < STAG_FP64 || p.precision > STAG_FP16_RU)
        return set_error(STAG_EINVAL, "stag_md_trajectory: mass, eps, tol > 0, nsteps, maxiter >= 1, a known "
                                      "precision and a finite beta are required");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    DeviceGuard dg(c->device);
    return md_trajectory(c, dims, links, momenta, phi, p, pick_stream(ctx, stream), info);
    STAG_GUARD_END
}

int stag_cg_solve_noalloc(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params, const double *b, double *x,
                          double *y, void *stream, stag_cg_info *info)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !params || !b || !x)
        return set_error(STAG_EINVAL, "stag_cg_solve_noalloc: NULL argument");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    int rc = validate_cg_params(*params);
    if (rc != STAG_OK)
        return rc;
    size_t dev_bytes = 0, host_bytes = 0;
    void *dev = noalloc_scratch(c->device, &dev_bytes);
    void *host = noalloc_host(c->device, &host_bytes);
    if (!dev || !host)
        return set_error(STAG_EHIP, "stag_cg_solve_noalloc: no fixed workspace on device %d", c->device);
    DeviceGuard dg(c->device);
    std::lock_guard<std::mutex> lk(noalloc_lock(c->device));
    return cg_solve_fixed(c, f, params, b, x, y, pick_stream(ctx, stream), info, dev, dev_bytes, host, host_bytes);
    STAG_GUARD_END
}

int stag_cg_solve_batch(stag_ctx *ctx, int32_t gauge_id, int32_t nrhs, const stag_cg_params *params,
                        const double *const *b, double *const *x, void *stream, stag_cg_info *infos)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !params || !b || !x || nrhs <= 0)
        return set_error(STAG_EINVAL, "stag_cg_solve_batch: NULL argument or nrhs <= 0");
    if (nrhs > 64)
        return set_error(STAG_EINVAL, "stag_cg_solve_batch: at most 64 right-hand sides");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    for (int i = 0; i < nrhs; ++i) {
        int rc = validate_cg_params(params[i]);
        if (rc != STAG_OK)
            return rc;
    }
    DeviceGuard dg(c->device);
    return cg_solve_batch(c, f, nrhs, params, b, x, nullptr, pick_stream(ctx, stream), infos);
    STAG_GUARD_END
}

int stag_tune_info(stag_ctx *ctx, int32_t gauge_id, int32_t precision, int32_t nrhs, int32_t *lanes_per_site,
                   int32_t *block, int32_t *rhs_tile, int32_t *use_tables)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || precision < 0 || precision > 2 || nrhs <= 0)
        return set_error(STAG_EINVAL, "stag_tune_info: bad argument");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    DeviceGuard dg(c->device);
    KernelCfg k = tune_config(c, f.get(), precision, nrhs, c->stream);
    if (lanes_per_site)
        *lanes_per_site = k.lps;
    if (block)
        *block = k.block;
    if (rhs_tile)
        *rhs_tile = k.rtile;
    if (use_tables)
        *use_tables = k.tables;
    return STAG_OK;
    STAG_GUARD_END
}

int stag_cg_tune_info(stag_ctx *ctx, int32_t gauge_id, int32_t precision, int32_t nrhs, int32_t *lanes_per_site,
                      int32_t *block, int32_t *rhs_tile, int32_t *use_tables, int32_t *reduce, int32_t *shared_links)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || precision < 0 || precision > 2 || nrhs <= 0)
        return set_error(STAG_EINVAL, "stag_cg_tune_info: bad argument");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    KernelCfg k;
    bool red = false;
    if (!cg_tuned_shape(c, f.get(), precision, nrhs, k, red))
        return set_error(STAG_ENOENT, "no CG solve with %d right-hand side(s) at precision %d has run on gauge id %d",
                         nrhs, precision, gauge_id);
    if (lanes_per_site)
        *lanes_per_site = k.lps;
    if (block)
        *block = k.block;
    if (rhs_tile)
        *rhs_tile = k.rtile;
    if (use_tables)
        *use_tables = k.tables;
    if (reduce)
        *reduce = red ? 1 : 0;
    if (shared_links)
        *shared_links = k.shared;
    return STAG_OK;
    STAG_GUARD_END
}

// ---- serving ------------------------------------------------------------------

static Server *server_of(Ctx *c)
{
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->server)
        c->server.reset(new Server(c));
    return c->server.get();
}

int stag_serve_config(stag_ctx *ctx, int32_t slots_per_field, int32_t epoch_iters, int32_t queue_capacity)
{
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (slots_per_field < 1 || slots_per_field > 64 || epoch_iters < 1 || epoch_iters > 1024 || queue_capacity < 1)
        return set_error(STAG_EINVAL, "stag_serve_config: slots 1..64, epoch 1..1024, capacity >= 1");
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->server)
        return set_error(STAG_EBUSY, "stag_serve_config: serving already started");
    c->slots_per_field = slots_per_field;
    c->epoch_iters = epoch_iters;
    c->queue_capacity = queue_capacity;
    return STAG_OK;
}

int stag_submit(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params, const double *b_dev, double *x_dev,
                uint64_t *ticket)
{
    STAG_GUARD_BEGIN
    clear_error();
    if (!ctx || !params || !b_dev || !x_dev || !ticket)
        return set_error(STAG_EINVAL, "stag_submit: NULL argument");
    int rc = validate_cg_params(*params);
    if (rc != STAG_OK)
        return rc;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    auto f = c->field(gauge_id);
    if (!f)
        return set_error(STAG_ENOENT, "unknown gauge id %d", gauge_id);
    if (f->kind != FIELD_STAGGERED)
        return set_error(STAG_EINVAL, "gauge id %d holds Wilson-fermion links", gauge_id);
    return server_of(c)->submit(f, *params, b_dev, x_dev, ticket);
    STAG_GUARD_END
}

int stag_poll(stag_ctx *ctx, uint64_t ticket, stag_cg_info *info)
{
    STAG_GUARD_BEGIN
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    return server_of(reinterpret_cast<Ctx *>(ctx))->poll(ticket, info, false);
    STAG_GUARD_END
}

int stag_wait(stag_ctx *ctx, uint64_t ticket, stag_cg_info *info)
{
    STAG_GUARD_BEGIN
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    return server_of(reinterpret_cast<Ctx *>(ctx))->poll(ticket, info, true);
    STAG_GUARD_END
}

int stag_release_ticket(stag_ctx *ctx, uint64_t ticket)
{
    STAG_GUARD_BEGIN
    if (!ctx)
        return set_error(STAG_EINVAL, "NULL context");
    return server_of(reinterpret_cast<Ctx *>(ctx))->release(ticket);
    STAG_GUARD_END
}

}  // extern "C"
