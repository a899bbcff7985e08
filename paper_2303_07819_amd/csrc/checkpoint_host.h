// Save and restore of a simulation (Algorithm 1 ends by saving the data of
// the run): everything a later sp_step reads, so that a run restored from a
// file continues exactly as the saved one would have.
//
// File layout (host byte order, no padding between records):
//   CkHeader;
//   counts   i32 [ncells]
//   xi, yi   u32 [n] each;  u, v, w, th, r, h  f32 [n] each
//   Q        f64 [4][ncells]   continuum state of the current level or, while
//                              the update of the last step is pending, of the
//                              level before it, followed by that step's
//                              statistics f64 [ncells][kMomStride]
//   contacts u64 [ncells];  cands u64 [ncells]   counters since the floes were set
//   vdisp    f32 [ncells]      displacement bound of the candidate lists
//   vcount   u8  [n];  vlist u16 [n * kListCap]   candidate lists
//   red      f64 [ncells][4]   reduced DEM of every cell (closure)
//   with SP_TANGENTIAL_SPRING: tsp_j u16x8 [n], tsp_x f64 [n][SP_SPRING_CAP]
// The grid, constants, flags and schedule of the loading context must equal
// the saved ones; the ocean is restored from the file.
#pragma once

namespace {

constexpr char kCkMagic[8] = {'S', 'P', 'D', 'E', 'M', 'C', 'K', '1'};

struct CkHeader {
    char magic[8];
    uint32_t version;
    uint32_t flags;
    int32_t nx, ny;
    int32_t schedule;
    int32_t kListCapSaved;
    double cell_lx, cell_ly, rho_ice, rho_ocean, cd, E, G, mu;
    int64_t n;
    int64_t kstep, steps, blk_steps;
    double t_now;
    float r_bin, skin, skin_set;
    int32_t nbx, nby, sched;
    uint64_t cfl_bits;
    double u0, v0;
    int32_t nmodes;
    int32_t spring_cap;
    int32_t lf_pending;         // the continuum update of level kstep - 1 is still to run
    int32_t pad;
    double lf_dt;
    double kx[SP_MAX_MODES], ky[SP_MAX_MODES], au[SP_MAX_MODES], av[SP_MAX_MODES], ph[SP_MAX_MODES];
};

struct CkFile {
    FILE* f = nullptr;
    ~CkFile()
    {
        if (f) fclose(f);
    }
};

template <class T>
bool ck_write(FILE* f, const std::vector<T>& v)
{
    return v.empty() || fwrite(v.data(), sizeof(T), v.size(), f) == v.size();
}

template <class T>
bool ck_read(FILE* f, std::vector<T>& v)
{
    return v.empty() || fread(v.data(), sizeof(T), v.size(), f) == v.size();
}

template <class T>
sp_status ck_d2h(sp_ctx* c, std::vector<T>& v, const void* src)
{
    if (!v.empty()) HIP_TRY(c, hipMemcpyAsync(v.data(), src, v.size() * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    return SP_OK;
}

template <class T>
sp_status ck_h2d(sp_ctx* c, void* dst, const std::vector<T>& v)
{
    if (!v.empty()) HIP_TRY(c, hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return SP_OK;
}

bool ck_same_params(const CkHeader& h, const sp_params& p)
{
    return h.nx == p.nx && h.ny == p.ny && h.cell_lx == p.cell_lx && h.cell_ly == p.cell_ly &&
           h.rho_ice == p.rho_ice && h.rho_ocean == p.rho_ocean && h.cd == p.cd && h.E == p.E && h.G == p.G &&
           h.mu == p.mu && h.flags == p.flags && h.schedule == p.schedule;
}

}  // namespace

extern "C" {

sp_status sp_save(sp_ctx* c, const char* path)
{
    if (!c) return SP_EINVAL;
    if (!path) return fail(c, SP_EINVAL, "null path");
    if (!c->have_floes) return fail(c, SP_ESTATE, "sp_save before sp_set_floes");
    if (c->hyb) return fail(c, SP_ESTATE, "sp_save with an active hybrid (its modes are not saved)");
    if (c->N0 > 1) return fail(c, SP_ESTATE, "sp_save runs at the cadence N0 = 1");
    // a pending continuum update is saved as pending (its operands with it),
    // so that the restored run takes it inside its next DEM launch as the
    // saved one would
    SP_TRY(join_block_lf(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    SP_TRY(check_device_err(c));

    CkHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kCkMagic, 8);
    h.version = 1;
    h.flags = c->p.flags;
    h.nx = c->p.nx;
    h.ny = c->p.ny;
    h.schedule = c->p.schedule;
    h.kListCapSaved = kListCap;
    h.cell_lx = c->p.cell_lx;
    h.cell_ly = c->p.cell_ly;
    h.rho_ice = c->p.rho_ice;
    h.rho_ocean = c->p.rho_ocean;
    h.cd = c->p.cd;
    h.E = c->p.E;
    h.G = c->p.G;
    h.mu = c->p.mu;
    h.n = c->n;
    h.kstep = c->kstep;
    h.steps = c->steps;
    h.blk_steps = c->blk_steps;
    h.t_now = c->t_now;
    h.r_bin = c->r_bin;
    h.skin = c->skin;
    h.skin_set = c->skin_set;
    h.nbx = c->nbx;
    h.nby = c->nby;
    h.sched = c->sched;
    h.u0 = c->u0;
    h.v0 = c->v0;
    h.nmodes = c->nmodes;
    h.spring_cap = SP_SPRING_CAP;
    h.lf_pending = c->lf_pending ? 1 : 0;
    h.lf_dt = c->lf_dt;
    for (int m = 0; m < c->nmodes; ++m) {
        h.kx[m] = c->kx[m];
        h.ky[m] = c->ky[m];
        h.au[m] = c->au[m];
        h.av[m] = c->av[m];
        h.ph[m] = c->ph[m];
    }
    HIP_TRY(c, hipMemcpyAsync(&h.cfl_bits, c->cfl_bits_d, 8, hipMemcpyDeviceToHost, c->stream));

    const size_t N = (size_t)c->n, NC = (size_t)c->ncells;
    std::vector<uint32_t> xi(N), yi(N);
    std::vector<float> fl[6] = {std::vector<float>(N), std::vector<float>(N), std::vector<float>(N),
                                std::vector<float>(N), std::vector<float>(N), std::vector<float>(N)};
    std::vector<double> Q(4 * NC), red(4 * NC, 0.0);
    std::vector<double> mprev(h.lf_pending ? NC * kMomStride : 0);
    std::vector<unsigned long long> contacts(NC), cands(NC);
    std::vector<float> vdisp(NC);
    std::vector<uint8_t> vcount(N);
    std::vector<uint16_t> vlist(N * kListCap);
    const bool spring = (c->p.flags & SP_TANGENTIAL_SPRING) != 0;
    std::vector<uint4> tj(spring ? N : 0);
    std::vector<double> tx(spring ? N * SP_SPRING_CAP : 0);
    const int64_t lvl = h.lf_pending ? c->kstep - 1 : c->kstep;   // level of the saved coarse state
    SP_TRY(ck_d2h(c, xi, c->xi));
    SP_TRY(ck_d2h(c, yi, c->yi));
    const void* fsrc[6] = {c->u, c->v, c->w, c->th, c->r, c->h};
    for (int k = 0; k < 6; ++k) SP_TRY(ck_d2h(c, fl[k], fsrc[k]));
    SP_TRY(ck_d2h(c, Q, c->Q[lvl & 1]));
    if (h.lf_pending) SP_TRY(ck_d2h(c, mprev, c->momb[lvl & 1]));
    SP_TRY(ck_d2h(c, contacts, c->contacts_d));
    SP_TRY(ck_d2h(c, cands, c->cands_d));
    SP_TRY(ck_d2h(c, vdisp, c->vdisp));
    SP_TRY(ck_d2h(c, vcount, c->vcount));
    SP_TRY(ck_d2h(c, vlist, c->vlist));
    if (c->red) SP_TRY(ck_d2h(c, red, c->red));
    if (spring) {
        SP_TRY(ck_d2h(c, tj, c->tsp_j));
        SP_TRY(ck_d2h(c, tx, c->tsp_x));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));

    CkFile f;
    f.f = fopen(path, "wb");
    if (!f.f) return fail(c, SP_EINVAL, "cannot open %s for writing", path);
    bool ok = fwrite(&h, sizeof h, 1, f.f) == 1;
    ok = ok && ck_write(f.f, c->counts_h) && ck_write(f.f, xi) && ck_write(f.f, yi);
    for (int k = 0; k < 6; ++k) ok = ok && ck_write(f.f, fl[k]);
    ok = ok && ck_write(f.f, Q) && ck_write(f.f, mprev) && ck_write(f.f, contacts) && ck_write(f.f, cands) && ck_write(f.f, vdisp) &&
         ck_write(f.f, vcount) && ck_write(f.f, vlist) && ck_write(f.f, red);
    if (spring) ok = ok && ck_write(f.f, tj) && ck_write(f.f, tx);
    ok = fclose(f.f) == 0 && ok;
    f.f = nullptr;
    if (!ok) return fail(c, SP_EDEVICE, "writing %s failed", path);
    return SP_OK;
}

sp_status sp_load(sp_ctx* c, const char* path)
{
    if (!c) return SP_EINVAL;
    if (!path) return fail(c, SP_EINVAL, "null path");
    CkFile f;
    f.f = fopen(path, "rb");
    if (!f.f) return fail(c, SP_EINVAL, "cannot open %s", path);
    CkHeader h;
    if (fread(&h, sizeof h, 1, f.f) != 1 || memcmp(h.magic, kCkMagic, 8) != 0 || h.version != 1)
        return fail(c, SP_EINVAL, "%s is not a saved simulation", path);
    if (!ck_same_params(h, c->p)) return fail(c, SP_EINVAL, "%s was saved with another grid, constants or flags", path);
    if (h.kListCapSaved != kListCap || h.spring_cap != SP_SPRING_CAP || h.n < 0 || h.n > INT32_MAX ||
        h.nmodes < 0 || h.nmodes > SP_MAX_MODES || (h.lf_pending && h.kstep < 1))
        return fail(c, SP_EINVAL, "%s: unsupported sizes", path);
    const size_t N = (size_t)h.n, NC = (size_t)c->ncells;
    std::vector<int32_t> counts(NC);
    std::vector<uint32_t> xi(N), yi(N);
    std::vector<float> fl[6] = {std::vector<float>(N), std::vector<float>(N), std::vector<float>(N),
                                std::vector<float>(N), std::vector<float>(N), std::vector<float>(N)};
    std::vector<double> Q(4 * NC), red(4 * NC);
    std::vector<double> mprev(h.lf_pending ? NC * kMomStride : 0);
    std::vector<unsigned long long> contacts(NC), cands(NC);
    std::vector<float> vdisp(NC);
    std::vector<uint8_t> vcount(N);
    std::vector<uint16_t> vlist(N * kListCap);
    const bool spring = (c->p.flags & SP_TANGENTIAL_SPRING) != 0;
    std::vector<uint4> tj(spring ? N : 0);
    std::vector<double> tx(spring ? N * SP_SPRING_CAP : 0);
    bool ok = ck_read(f.f, counts) && ck_read(f.f, xi) && ck_read(f.f, yi);
    for (int k = 0; k < 6; ++k) ok = ok && ck_read(f.f, fl[k]);
    ok = ok && ck_read(f.f, Q) && ck_read(f.f, mprev) && ck_read(f.f, contacts) && ck_read(f.f, cands) && ck_read(f.f, vdisp) &&
         ck_read(f.f, vcount) && ck_read(f.f, vlist) && ck_read(f.f, red);
    if (spring) ok = ok && ck_read(f.f, tj) && ck_read(f.f, tx);
    if (!ok) return fail(c, SP_EINVAL, "%s is truncated", path);
    fclose(f.f);
    f.f = nullptr;

    // ocean, then the floes (buckets, schedule, statistics, buffers)
    SP_TRY(sp_set_ocean(c, h.u0, h.v0, h.nmodes, h.kx, h.ky, h.au, h.av, h.ph));
    SP_TRY(sp_set_floes(c, h.n, counts.data(), xi.data(), yi.data(), fl[0].data(), fl[1].data(), fl[2].data(),
                        fl[3].data(), fl[4].data(), fl[5].data()));
    // the contact search as it was (re-synchronised radii may differ from the
    // radii the sub-bins were sized for)
    if (c->r_bin != h.r_bin) {
        SP_TRY(plan_bins(c, h.r_bin, h.n > 0));
        SP_TRY(prepare_buckets(c));
    }
    if (c->nbx != h.nbx || c->nby != h.nby || c->sched != h.sched)
        return fail(c, SP_EINVAL, "%s: contact search cannot be restored", path);
    c->skin = h.skin;
    c->skin_set = h.skin_set;
    // the continuum at the saved level (both buffers), counters, lists,
    // reduced DEMs and contact history
    c->kstep = h.kstep;
    c->steps = h.steps;
    c->blk_steps = h.blk_steps;
    c->t_now = h.t_now;
    SP_TRY(ck_h2d(c, c->Q[0], Q));
    SP_TRY(ck_h2d(c, c->Q[1], Q));
    if (h.lf_pending) {   // the update of level kstep - 1, from its statistics
        const int64_t lvl = h.kstep - 1;
        SP_TRY(ck_h2d(c, c->momb[lvl & 1], mprev));
        c->lf_pending = true;
        c->lf_dt = h.lf_dt;
    } else {
        c->lf_pending = false;
    }
    SP_TRY(ck_h2d(c, c->contacts_d, contacts));
    SP_TRY(ck_h2d(c, c->cands_d, cands));
    SP_TRY(ck_h2d(c, c->vdisp, vdisp));
    SP_TRY(ck_h2d(c, c->vcount, vcount));
    SP_TRY(ck_h2d(c, c->vlist, vlist));
    if (c->red) SP_TRY(ck_h2d(c, c->red, red));
    if (spring) {
        SP_TRY(ck_h2d(c, c->tsp_j, tj));
        SP_TRY(ck_h2d(c, c->tsp_x, tx));
    }
    HIP_TRY(c, hipMemcpyAsync(c->cfl_bits_d, &h.cfl_bits, 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SP_OK;
}

sp_status sp_get_size(sp_ctx* c, int64_t* nfloes, int32_t* ncells)
{
    if (!c) return SP_EINVAL;
    if (nfloes) *nfloes = c->have_floes ? c->n : 0;
    if (ncells) *ncells = c->ncells;
    return SP_OK;
}

}  // extern "C"
