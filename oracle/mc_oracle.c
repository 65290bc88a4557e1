/*
 * mc_oracle.c -- plain FP64 CPU oracle for single-spin Metropolis sweeps of the
 * classical anisotropic Heisenberg model (Charilaou, "GPU-accelerated Monte Carlo
 * simulations of anisotropic Heisenberg ferromagnets", arXiv:2106.11286).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the GPU
 * library.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with the
 * HIP path: geometry comes from brute-force distance tests, neighbours from an
 * explicit list, energies from an explicit bond list.
 *
 * What it computes (paper references are to equations / paragraphs):
 *   H = -J sum_<ij> S_i.S_j - K sum_i (S_i.e)^2            Eq. (1)
 *   with nearest-neighbour bonds, each unordered pair counted once.
 *   Metropolis single-spin update (pick, propose, accept if dH <= 0 or
 *   P <= exp(-beta dH)), as in the paragraph introducing the Metropolis method.
 *   Magnetisation vector M = sum_i S_i / (N |S|)             Eq. (2)
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - spins are visited colour by colour (colour c = 0..C-1), every site of a
 *     colour in ascending canonical index; no bond joins two sites of the same
 *     colour, so the order inside a colour cannot change the result;
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = (seed lo32, seed hi32), counter = (site s, replica id, sweep t, tag);
 *     tag 0 = Metropolis move, 1 = initial state;
 *   - a uniform u in (0,1) uses the top 23 bits of a word: u = (k + 1/2) 2^-23,
 *     exactly representable in binary32 and binary64;
 *   - proposal: z = 2 u0 - 1, phi = 2 pi u1, S' = (sqrt(1-z^2) cos phi,
 *     sqrt(1-z^2) sin phi, z), uniform on the unit sphere; P = u2;
 *   - accept iff dH <= 0, or T > 0 and P <= exp(-dH/T); T = +inf means beta = 0;
 *   - an accepted spin is stored as S'/|S'|.
 *
 * Parallelism: OpenMP over the sites of one colour only.  Results do not depend
 * on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, written from the published description (SC'11, Sec. 4):     */
/* two 32x32->64 products per round, the high halves xored with the other two */
/* counter words and the key, the key bumped by the Weyl constants.           */
/* ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits of a 32-bit word: (k + 1/2) * 2^-23. */
double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Uniform point on the unit sphere from two uniforms (Archimedes: z is uniform
 * on [-1,1], the azimuth uniform on [0, 2 pi)).  Proposal step of the
 * Metropolis paragraph: the new orientation is drawn independently of the old. */
void orc_sphere_point(double u0, double u1, double out[3])
{
    double z = 2.0 * u0 - 1.0;
    double phi = 2.0 * M_PI * u1;
    double r = sqrt(1.0 - z * z);
    out[0] = r * cos(phi);
    out[1] = r * sin(phi);
    out[2] = z;
}

/* ------------------------------------------------------------------------- */
/* Lattice: explicit site table, neighbour lists and colour per site.         */
/* ------------------------------------------------------------------------- */
enum { ORC_SC = 0, ORC_BCC = 1, ORC_FCC = 2 };
/* neighbour-list stride: the coordination number of the lattice kind */
static int zmax_of(int kind) { return kind == 0 ? 6 : (kind == 1 ? 8 : 12); }

typedef struct {
    int kind, Lx, Ly, Lz, nb;          /* nb = basis sites per cubic cell    */
    uint32_t periodic_mask;            /* bit0 x, bit1 y, bit2 z             */
    double sphere_radius;              /* <= 0: whole box                    */
    int64_t n_box;                     /* Lx*Ly*Lz*nb                        */
    int64_t n_occ;                     /* occupied sites                     */
    int n_colours;
    uint8_t *occ;                      /* [n_box]                            */
    uint8_t *colour;                   /* [n_box]                            */
    int8_t *nnb;                       /* [n_box] neighbour count            */
    int zmax;                          /* stride of nbr                      */
    int32_t *nbr;                      /* [n_box][zmax] canonical indices    */
    int64_t n_bonds;                   /* unordered pairs, with multiplicity */
    int same_colour_bonds;             /* must be 0 for a valid colouring    */
} orc_lattice;

/* basis positions in units of the cubic cell, times 2 (so they are integers) */
static const int BASIS2_SC[1][3] = {{0, 0, 0}};
static const int BASIS2_BCC[2][3] = {{0, 0, 0}, {1, 1, 1}};
static const int BASIS2_FCC[4][3] = {{0, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};

static const int (*basis2_of(int kind))[3]
{
    if (kind == ORC_SC) return BASIS2_SC;
    if (kind == ORC_BCC) return BASIS2_BCC;
    return BASIS2_FCC;
}

static int nbasis_of(int kind) { return kind == ORC_SC ? 1 : (kind == ORC_BCC ? 2 : 4); }

/* squared nearest-neighbour distance in (half-cell units)^2:
 * sc 1 cell -> 4; bcc sqrt(3)/2 -> 3; fcc 1/sqrt(2) -> 2 */
static int nn_dist2_half(int kind) { return kind == ORC_SC ? 4 : (kind == ORC_BCC ? 3 : 2); }

int64_t orc_site_index(const orc_lattice *L, int x, int y, int z, int b)
{
    return (((int64_t)z * L->Ly + y) * L->Lx + x) * L->nb + b;
}

/* Occupancy: inside a sphere of the given radius (in cells) centred at the box
 * centre (Lx/2, Ly/2, Lz/2), or the whole box.  Distances in half-cell units
 * are integers, so the test is exact. */
static int site_occupied(const orc_lattice *L, int x, int y, int z, int b)
{
    if (L->sphere_radius <= 0.0) return 1;
    const int (*B)[3] = basis2_of(L->kind);
    int64_t qx = 2 * (int64_t)x + B[b][0] - L->Lx;
    int64_t qy = 2 * (int64_t)y + B[b][1] - L->Ly;
    int64_t qz = 2 * (int64_t)z + B[b][2] - L->Lz;
    double q = (double)(qx * qx + qy * qy + qz * qz);
    return q <= 4.0 * L->sphere_radius * L->sphere_radius;
}

static int site_colour(const orc_lattice *L, int x, int y, int z, int b)
{
    if (L->kind == ORC_SC) return (x + y + z) & 1;
    return b;
}

void orc_lattice_free(orc_lattice *L)
{
    if (!L) return;
    free(L->occ); free(L->colour); free(L->nnb); free(L->nbr);
    free(L);
}

/* Nearest neighbours of site (x, y, z, b) by brute force: every basis site of
 * the 27 surrounding cells at the nearest-neighbour distance, wrapping
 * periodic axes and dropping open-face and unoccupied sites.  They are listed
 * in loop order (dz, dy, dx, b') ascending, which fixes the summation order of
 * the local field.  Returns the count, or -1 if it exceeds the coordination. */
static int neighbours_of(const orc_lattice *L, int x, int y, int z, int b, int32_t *out)
{
    const int (*B)[3] = basis2_of(L->kind);
    const int d2nn = nn_dist2_half(L->kind);
    const int dims[3] = {L->Lx, L->Ly, L->Lz};
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                for (int b2 = 0; b2 < L->nb; ++b2) {
                    int ex = 2 * dx + B[b2][0] - B[b][0];
                    int ey = 2 * dy + B[b2][1] - B[b][1];
                    int ez = 2 * dz + B[b2][2] - B[b][2];
                    if (ex * ex + ey * ey + ez * ez != d2nn) continue;
                    int c[3] = {x + dx, y + dy, z + dz};
                    int ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        if (c[a] < 0 || c[a] >= dims[a]) {
                            if (L->periodic_mask & (1u << a))
                                c[a] = (c[a] + dims[a]) % dims[a];
                            else
                                ok = 0;
                        }
                    }
                    if (!ok) continue;
                    if (!site_occupied(L, c[0], c[1], c[2], b2)) continue;
                    if (cnt >= L->zmax) return -1;
                    out[cnt++] = (int32_t)orc_site_index(L, c[0], c[1], c[2], b2);
                }
    return cnt;
}

/* Build the lattice: site table, colours and the neighbour list of every
 * occupied site (see neighbours_of). */
orc_lattice *orc_lattice_new(int kind, int Lx, int Ly, int Lz, uint32_t periodic_mask,
                             double sphere_radius)
{
    if (kind < 0 || kind > 2 || Lx < 1 || Ly < 1 || Lz < 1) return NULL;
    if ((double)Lx * Ly * Lz * nbasis_of(kind) >= 2147483647.0) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    L->kind = kind; L->Lx = Lx; L->Ly = Ly; L->Lz = Lz;
    L->nb = nbasis_of(kind);
    L->periodic_mask = periodic_mask;
    L->sphere_radius = sphere_radius;
    L->n_box = (int64_t)Lx * Ly * Lz * L->nb;
    L->n_colours = kind == ORC_SC ? 2 : L->nb;
    L->occ = (uint8_t *)malloc((size_t)L->n_box);
    L->colour = (uint8_t *)malloc((size_t)L->n_box);
    L->nnb = (int8_t *)calloc((size_t)L->n_box, 1);
    L->zmax = zmax_of(kind);
    L->nbr = (int32_t *)malloc((size_t)L->n_box * L->zmax * sizeof(int32_t));
    if (!L->occ || !L->colour || !L->nnb || !L->nbr) { orc_lattice_free(L); return NULL; }

    int64_t n_occ = 0;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x)
                for (int b = 0; b < L->nb; ++b) {
                    int64_t s = orc_site_index(L, x, y, z, b);
                    L->occ[s] = (uint8_t)site_occupied(L, x, y, z, b);
                    L->colour[s] = (uint8_t)site_colour(L, x, y, z, b);
                    n_occ += L->occ[s];
                }
    L->n_occ = n_occ;

    int64_t n_half_bonds = 0;
    int same = 0;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x)
                for (int b = 0; b < L->nb; ++b) {
                    int64_t s = orc_site_index(L, x, y, z, b);
                    if (!L->occ[s]) continue;
                    int cnt = neighbours_of(L, x, y, z, b, L->nbr + s * L->zmax);
                    if (cnt < 0) { orc_lattice_free(L); return NULL; }
                    for (int k = 0; k < cnt; ++k)
                        if (L->colour[L->nbr[s * L->zmax + k]] == L->colour[s]) same = 1;
                    L->nnb[s] = (int8_t)cnt;
                    n_half_bonds += cnt;
                }
    L->n_bonds = n_half_bonds / 2;
    L->same_colour_bonds = same;
    return L;
}

/* Geometry only (no tables): for evaluating single sites of lattices too
 * large to tabulate.  Free with orc_lattice_free. */
orc_lattice *orc_geometry_new(int kind, int Lx, int Ly, int Lz, uint32_t periodic_mask,
                              double sphere_radius)
{
    if (kind < 0 || kind > 2 || Lx < 1 || Ly < 1 || Lz < 1) return NULL;
    if ((double)Lx * Ly * Lz * nbasis_of(kind) >= 2147483647.0) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    L->kind = kind; L->Lx = Lx; L->Ly = Ly; L->Lz = Lz;
    L->nb = nbasis_of(kind);
    L->periodic_mask = periodic_mask;
    L->sphere_radius = sphere_radius;
    L->n_box = (int64_t)Lx * Ly * Lz * L->nb;
    L->n_colours = kind == ORC_SC ? 2 : L->nb;
    L->zmax = zmax_of(kind);
    L->n_occ = -1;
    L->n_bonds = -1;
    return L;
}

/* accessors for the Python side */
int64_t orc_lattice_n_box(const orc_lattice *L) { return L->n_box; }
int64_t orc_lattice_n_occ(const orc_lattice *L) { return L->n_occ; }
int64_t orc_lattice_n_bonds(const orc_lattice *L) { return L->n_bonds; }
int orc_lattice_n_colours(const orc_lattice *L) { return L->n_colours; }
int orc_lattice_same_colour_bonds(const orc_lattice *L) { return L->same_colour_bonds; }
int orc_lattice_zmax(const orc_lattice *L) { return L->zmax; }
void orc_lattice_tables(const orc_lattice *L, uint8_t *occ, uint8_t *colour, int8_t *nnb,
                        int32_t *nbr)
{
    if (occ) memcpy(occ, L->occ, (size_t)L->n_box);
    if (colour) memcpy(colour, L->colour, (size_t)L->n_box);
    if (nnb) memcpy(nnb, L->nnb, (size_t)L->n_box);
    if (nbr) memcpy(nbr, L->nbr, (size_t)L->n_box * L->zmax * sizeof(int32_t));
}

/* ------------------------------------------------------------------------- */
/* Model parameters                                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    double J, K, e[3], T;
    uint64_t seed;
    uint32_t replica_id;
} orc_params;

static void unit_axis(const double e_in[3], double e[3])
{
    double n = sqrt(e_in[0] * e_in[0] + e_in[1] * e_in[1] + e_in[2] * e_in[2]);
    e[0] = e_in[0] / n; e[1] = e_in[1] / n; e[2] = e_in[2] / n;
}

static void philox_site(uint64_t seed, uint32_t s, uint32_t rid, uint32_t t, uint32_t tag,
                        uint32_t out[4])
{
    uint32_t ctr[4] = {s, rid, t, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Initial state.  mode 0: uniform on the sphere from Philox (tag 1, sweep 0);
 * mode 1: every spin along the easy axis e.  Unoccupied sites hold zero. */
void orc_init(const orc_lattice *L, const orc_params *p, int mode, double *sx, double *sy,
              double *sz)
{
    double e[3];
    unit_axis(p->e, e);
    for (int64_t s = 0; s < L->n_box; ++s) {
        if (!L->occ[s]) { sx[s] = sy[s] = sz[s] = 0.0; continue; }
        if (mode == 1) { sx[s] = e[0]; sy[s] = e[1]; sz[s] = e[2]; continue; }
        uint32_t w[4];
        philox_site(p->seed, (uint32_t)s, p->replica_id, 0u, 1u, w);
        double v[3];
        orc_sphere_point(orc_uniform(w[0]), orc_uniform(w[1]), v);
        sx[s] = v[0]; sy[s] = v[1]; sz[s] = v[2];
    }
}

/* Energy change of replacing S by Sn at one site with local field h = J sum S_j:
 * from Eq. (1), dH = -h.(Sn - S) - K[(Sn.e)^2 - (S.e)^2]. */
double orc_delta_h(const double h[3], const double S[3], const double Sn[3], double K,
                   const double e[3])
{
    double dex = -(h[0] * (Sn[0] - S[0]) + h[1] * (Sn[1] - S[1]) + h[2] * (Sn[2] - S[2]));
    double pn = Sn[0] * e[0] + Sn[1] * e[1] + Sn[2] * e[2];
    double po = S[0] * e[0] + S[1] * e[1] + S[2] * e[2];
    return dex - K * (pn * pn - po * po);
}

/* One Metropolis attempt (the three steps of the Metropolis paragraph) at
 * canonical site s with local field h = J sum_j S_j and current spin S.
 * Writes the proposal outcome: dH, the decision, beta*dH + ln P (accept iff
 * <= 0 when dH > 0) and the spin after the attempt. */
static int attempt(const orc_params *p, const double e[3], uint32_t t, uint32_t s,
                   const double h[3], const double S[3], double *dH_out, double *margin_out,
                   double S_after[3])
{
    const double beta = (p->T > 0.0) ? 1.0 / p->T : 0.0; /* T = +inf gives 0 */
    uint32_t w[4];
    philox_site(p->seed, s, p->replica_id, t, 0u, w);
    double Sn[3];
    orc_sphere_point(orc_uniform(w[0]), orc_uniform(w[1]), Sn);
    double P = orc_uniform(w[2]);
    double dH = orc_delta_h(h, S, Sn, p->K, e);
    int accept;
    if (dH <= 0.0) accept = 1;
    else if (p->T > 0.0) accept = (P <= exp(-beta * dH));
    else accept = 0;
    *dH_out = dH;
    *margin_out = beta * dH + log(P);
    if (accept) {
        double n = sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2]);
        S_after[0] = Sn[0] / n; S_after[1] = Sn[1] / n; S_after[2] = Sn[2] / n;
    } else {
        S_after[0] = S[0]; S_after[1] = S[1]; S_after[2] = S[2];
    }
    return accept;
}

/* One colour pass at sweep t: every occupied site of colour c gets one
 * Metropolis attempt.  Optional per-site outputs (indexed by canonical site;
 * untouched elsewhere): dH, the decision, and beta*dH + ln P.  Returns the
 * number accepted. */
int64_t orc_pass(const orc_lattice *L, const orc_params *p, int c, uint32_t t, double *sx,
                 double *sy, double *sz, double *out_dh, uint8_t *out_acc, double *out_margin)
{
    double e[3];
    unit_axis(p->e, e);
    int64_t n_acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_acc)
    for (int64_t s = 0; s < L->n_box; ++s) {
        if (!L->occ[s] || L->colour[s] != c) continue;
        double h[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < L->nnb[s]; ++k) {
            int64_t j = L->nbr[s * L->zmax + k];
            h[0] += sx[j]; h[1] += sy[j]; h[2] += sz[j];
        }
        h[0] *= p->J; h[1] *= p->J; h[2] *= p->J;
        double S[3] = {sx[s], sy[s], sz[s]}, Sa[3], dH, mg;
        int accept = attempt(p, e, t, (uint32_t)s, h, S, &dH, &mg, Sa);
        if (out_dh) out_dh[s] = dH;
        if (out_acc) out_acc[s] = (uint8_t)accept;
        if (out_margin) out_margin[s] = mg;
        if (accept) {
            sx[s] = Sa[0]; sy[s] = Sa[1]; sz[s] = Sa[2];
            n_acc += 1;
        }
    }
    return n_acc;
}

/* The attempt of one site at sweep t on a geometry without tables, for
 * lattices too large to tabulate: neighbours by brute force (neighbours_of),
 * spins in natural order.  out = {dH, accepted, beta*dH + ln P, S_after[3],
 * h[3]}.  Returns 0, or -1 for an unoccupied site or an invalid index. */
int orc_site_attempt(const orc_lattice *G, const orc_params *p, uint32_t t, const double *sx,
                     const double *sy, const double *sz, int64_t s, double out[9])
{
    if (s < 0 || s >= G->n_box) return -1;
    const int b = (int)(s % G->nb);
    const int64_t cell = s / G->nb;
    const int x = (int)(cell % G->Lx);
    const int y = (int)((cell / G->Lx) % G->Ly);
    const int z = (int)(cell / ((int64_t)G->Lx * G->Ly));
    if (!site_occupied(G, x, y, z, b)) return -1;
    int32_t nb[12];
    int cnt = neighbours_of(G, x, y, z, b, nb);
    if (cnt < 0) return -1;
    double e[3];
    unit_axis(p->e, e);
    double h[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < cnt; ++k) {
        h[0] += sx[nb[k]]; h[1] += sy[nb[k]]; h[2] += sz[nb[k]];
    }
    h[0] *= p->J; h[1] *= p->J; h[2] *= p->J;
    double S[3] = {sx[s], sy[s], sz[s]}, Sa[3], dH, mg;
    int accept = attempt(p, e, t, (uint32_t)s, h, S, &dH, &mg, Sa);
    out[0] = dH; out[1] = accept; out[2] = mg;
    out[3] = Sa[0]; out[4] = Sa[1]; out[5] = Sa[2];
    out[6] = h[0]; out[7] = h[1]; out[8] = h[2];
    return 0;
}

/* Observables of a state, from scratch, serial and in fixed order:
 * out = {Mx, My, Mz (sums, not normalised), E_exch, E_anis}.
 * E_exch sums every bond once (pair i<j taken from i's list). */
void orc_observables(const orc_lattice *L, const orc_params *p, const double *sx,
                     const double *sy, const double *sz, double out[5])
{
    double e[3];
    unit_axis(p->e, e);
    double mx = 0, my = 0, mz = 0, ex = 0, ea = 0;
    for (int64_t s = 0; s < L->n_box; ++s) {
        if (!L->occ[s]) continue;
        mx += sx[s]; my += sy[s]; mz += sz[s];
        double pe = sx[s] * e[0] + sy[s] * e[1] + sz[s] * e[2];
        ea += pe * pe;
        for (int k = 0; k < L->nnb[s]; ++k) {
            int64_t j = L->nbr[s * L->zmax + k];
            if (j > s) ex += sx[s] * sx[j] + sy[s] * sy[j] + sz[s] * sz[j];
        }
    }
    out[0] = mx; out[1] = my; out[2] = mz;
    out[3] = -p->J * ex;
    out[4] = -p->K * ea;
}

/* One sweep: colour passes 0..C-1 at sweep counter t.  Returns accepted moves. */
int64_t orc_sweep(const orc_lattice *L, const orc_params *p, uint32_t t, double *sx, double *sy,
                  double *sz)
{
    int64_t n = 0;
    for (int c = 0; c < L->n_colours; ++c) n += orc_pass(L, p, c, t, sx, sy, sz, NULL, NULL, NULL);
    return n;
}

/* n sweeps starting at counter t0.  If rec != NULL, after every sweep write
 * {Mx, My, Mz, E_exch, E_anis, n_acc} (6 doubles) to rec[6*i]. */
void orc_run(const orc_lattice *L, const orc_params *p, uint32_t t0, uint32_t n_sweeps,
             double *sx, double *sy, double *sz, double *rec)
{
    for (uint32_t i = 0; i < n_sweeps; ++i) {
        int64_t na = orc_sweep(L, p, t0 + i, sx, sy, sz);
        if (rec) {
            double o[5];
            orc_observables(L, p, sx, sy, sz, o);
            for (int k = 0; k < 5; ++k) rec[6 * (size_t)i + k] = o[k];
            rec[6 * (size_t)i + 5] = (double)na;
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
