/*
 * FP64 CPU oracle for the neural-volume hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library, and the HIP
 * library never calls it.
 *
 * It computes, plainly and slowly, what the paper's method computes:
 *   - a multi-resolution hash-grid encoding (Section 3.1, Fig. 1B): per level,
 *     the 8 corners of the enclosing grid cell are looked up in that level's
 *     table and trilinearly interpolated, and level features are concatenated;
 *   - a bias-free ReLU MLP on the concatenated features (Section 3.1), its
 *     output neuron either linear or, as an option, followed by a ReLU;
 *   - the sampling step (Section 4): uniform random coordinates in [0,1)^3
 *     with a trilinearly interpolated ground-truth value;
 *   - one optimisation step: L2 or L1 loss, analytic gradient, Adam with an
 *     exponentially decaying learning rate and L2 regularisation of the
 *     network weights (Section 3.1 and the appendix's default optimiser;
 *     Kingma and Ba 2014);
 *   - the ray-marched emission-absorption renderer fed by streamed samples
 *     (Section 5.2.1), with macro-cell value ranges built from training
 *     samples and empty-space skipping (Section 5.3);
 *   - decoding the whole grid and its PSNR (Section 6).
 *
 * Readings of the paper where it is silent (the hash, the resolution rule,
 * the sampler convention, the loss form, the camera and transfer function)
 * are listed at the top of the design notes; each function names the one it
 * uses.  Every floating-point value is FP64 except where noted (the ray
 * geometry, which is specified in binary32 and evaluated here with one
 * IEEE rounding per operation; build with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LEVELS 32

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea, Flood 2014).      */
/* Output n of stream (seed, stream) is the n-th output of a SplitMix64     */
/* sequence whose initial state is seed XOR (stream << 56).                 */
/* ------------------------------------------------------------------------ */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_rng_u64(uint64_t seed, uint32_t stream, uint64_t index)
{
    uint64_t s0 = seed ^ ((uint64_t)stream << 56);
    return orc_mix64(s0 + (index + 1ull) * 0x9E3779B97F4A7C15ull);
}

/* Uniform in [0,1): top 24 bits, exactly representable in binary32. */
double orc_rng_u01(uint64_t seed, uint32_t stream, uint64_t index)
{
    return (double)(orc_rng_u64(seed, stream, index) >> 40) * 0x1p-24;
}

/* ------------------------------------------------------------------------ */
/* Model description and parameter layout.                                  */
/*                                                                          */
/* desc = { L, F, log2T, width, n_hidden, out_relu, N_0, ..., N_{L-1} }     */
/* Level l is a grid of N_l vertices per axis spanning [0,1].  It is stored */
/* densely when N_l^3 <= T and hashed into T entries otherwise, so its      */
/* table has min(T, N_l^3) entries of F features (entry-major).  Tables     */
/* come first in level order; then the bias-free MLP matrices, row-major    */
/* [out][in]: [width][L*F], (n_hidden-1) x [width][width], [1][width].      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int L, F, log2T, width, n_hidden, n_in;
    int64_t T;
    int32_t N[ORC_MAX_LEVELS];
    int dense[ORC_MAX_LEVELS];
    int64_t size[ORC_MAX_LEVELS];
    int64_t off[ORC_MAX_LEVELS + 1];
    int64_t n_table, n_mlp, n_params;
    int n_layers;         /* n_hidden + 1 matrices */
    int out_relu;         /* 1: ReLU on the output neuron */
    int64_t w_off[16];    /* offset of each matrix, relative to the MLP block */
    int w_in[16], w_out[16];
} orc_model;

static int orc_model_from_desc(const int32_t* desc, orc_model* m)
{
    memset(m, 0, sizeof(*m));
    m->L = desc[0];
    m->F = desc[1];
    m->log2T = desc[2];
    m->width = desc[3];
    m->n_hidden = desc[4];
    m->out_relu = desc[5];
    if ((m->out_relu != 0 && m->out_relu != 1) || m->L < 1 || m->L > ORC_MAX_LEVELS || m->F < 1 || m->log2T < 1 || m->log2T > 30 ||
        m->width < 1 || m->n_hidden < 1 || m->n_hidden > 14)
        return -1;
    m->T = (int64_t)1 << m->log2T;
    m->n_in = m->L * m->F;
    m->off[0] = 0;
    for (int l = 0; l < m->L; ++l) {
        int64_t N = desc[6 + l];
        if (N < 2) return -1;
        m->N[l] = (int32_t)N;
        int64_t cube = N * N * N;
        m->dense[l] = cube <= m->T;
        m->size[l] = m->dense[l] ? cube : m->T;
        m->off[l + 1] = m->off[l] + m->size[l];
    }
    m->n_table = m->off[m->L] * m->F;
    m->n_layers = m->n_hidden + 1;
    int64_t pos = 0;
    for (int i = 0; i < m->n_layers; ++i) {
        m->w_in[i] = (i == 0) ? m->n_in : m->width;
        m->w_out[i] = (i == m->n_layers - 1) ? 1 : m->width;
        m->w_off[i] = pos;
        pos += (int64_t)m->w_in[i] * m->w_out[i];
    }
    m->n_mlp = pos;
    m->n_params = m->n_table + m->n_mlp;
    return 0;
}

/* Writes level sizes, level offsets (entries) and {n_table, n_mlp, n_params}. */
int orc_layout(const int32_t* desc, int64_t* size, int64_t* off, int64_t* counts)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m)) return -1;
    for (int l = 0; l < m.L; ++l) {
        size[l] = m.size[l];
        off[l] = m.off[l];
    }
    off[m.L] = m.off[m.L];
    counts[0] = m.n_table;
    counts[1] = m.n_mlp;
    counts[2] = m.n_params;
    return 0;
}

/*
 * Vertices per axis of each level: N_l = N_min * b^l.  When that is an
 * integer (within 1e-9 relative) it is used as is, otherwise rounded up.
 * If max_res > 0 the growth factor is b = exp((ln N_max - ln N_min)/(L-1)).
 */
int orc_resolutions(int L, int base, double scale, int max_res, int32_t* out)
{
    if (L < 1 || L > ORC_MAX_LEVELS || base < 2) return -1;
    double b = scale;
    if (max_res > 0) b = (L > 1) ? exp((log((double)max_res) - log((double)base)) / (double)(L - 1)) : 1.0;
    for (int l = 0; l < L; ++l) {
        double r = (double)base * pow(b, (double)l);
        double rr = floor(r + 0.5);
        out[l] = (int32_t)((fabs(r - rr) < 1e-9 * r) ? rr : ceil(r));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Encoding (Section 3.1, Fig. 1B).                                         */
/* ------------------------------------------------------------------------ */

/* Clamp a binary32 coordinate to [0,1]; NaN maps to 0. */
static double orc_clamp01f(float x)
{
    float y = fminf(fmaxf(x, 0.0f), 1.0f);
    return (double)y;
}

/*
 * Geometry of one level along one axis: p = x*(N-1) (exact in FP64 for a
 * binary32 x and N <= 2^24), cell c = min(floor(p), N-2), weight w = p - c.
 */
static void orc_axis(double x, int32_t N, int64_t* c, double* w)
{
    double p = x * (double)(N - 1);
    double fl = floor(p);
    if (fl > (double)(N - 2)) fl = (double)(N - 2);
    *c = (int64_t)fl;
    *w = p - fl;
}

/*
 * Table slot of vertex (vx,vy,vz) at a level: dense row-major index when the
 * level is dense, else the spatial hash of Mueller et al. 2022 (the encoding
 * the paper adopts), (vx*1 XOR vy*2654435761 XOR vz*805459861) mod 2^32,
 * reduced modulo T (a power of two).
 */
static uint32_t orc_slot(const orc_model* m, int l, int64_t vx, int64_t vy, int64_t vz)
{
    if (m->dense[l]) {
        int64_t N = m->N[l];
        return (uint32_t)(vx + N * (vy + N * vz));
    }
    uint32_t h = ((uint32_t)vx * 1u) ^ ((uint32_t)vy * 2654435761u) ^ ((uint32_t)vz * 805459861u);
    return h & (uint32_t)(m->T - 1);
}

/*
 * Corners of level l for one point: global entry index (level offset added)
 * and trilinear weight, corner order delta = (dx, dy, dz) with dx fastest.
 */
static void orc_corners(const orc_model* m, int l, const double x[3], int64_t idx[8], double wt[8])
{
    int64_t c[3];
    double w[3];
    for (int a = 0; a < 3; ++a) orc_axis(x[a], m->N[l], &c[a], &w[a]);
    for (int k = 0; k < 8; ++k) {
        int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        double wk = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
        idx[k] = m->off[l] + (int64_t)orc_slot(m, l, c[0] + dx, c[1] + dy, c[2] + dz);
        wt[k] = wk;
    }
}

static void orc_encode_one(const orc_model* m, const double* table, const float* xyz, double* e)
{
    double x[3] = {orc_clamp01f(xyz[0]), orc_clamp01f(xyz[1]), orc_clamp01f(xyz[2])};
    for (int l = 0; l < m->L; ++l) {
        int64_t idx[8];
        double wt[8];
        orc_corners(m, l, x, idx, wt);
        for (int f = 0; f < m->F; ++f) {
            double s = 0.0;
            for (int k = 0; k < 8; ++k) s += wt[k] * table[idx[k] * m->F + f];
            e[l * m->F + f] = s;
        }
    }
}

/* feat[n][L*F] = encoding of xyz[n][3] under the table part of params. */
int orc_encode(const int32_t* desc, const double* params, const float* xyz, int64_t n, double* feat)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) orc_encode_one(&m, params, xyz + 3 * i, feat + i * m.n_in);
    return 0;
}

/* idx[n][L][8] = slot within the level's table (no level offset); w[n][L][8]. */
int orc_encode_debug(const int32_t* desc, const float* xyz, int64_t n, uint32_t* idx, double* w)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x[3] = {orc_clamp01f(xyz[3 * i]), orc_clamp01f(xyz[3 * i + 1]), orc_clamp01f(xyz[3 * i + 2])};
        for (int l = 0; l < m.L; ++l) {
            int64_t g[8];
            double wt[8];
            orc_corners(&m, l, x, g, wt);
            for (int k = 0; k < 8; ++k) {
                idx[(i * m.L + l) * 8 + k] = (uint32_t)(g[k] - m.off[l]);
                w[(i * m.L + l) * 8 + k] = wt[k];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* MLP (Section 3.1): bias-free, ReLU on hidden layers; the output neuron    */
/* is linear, or followed by a ReLU (an option: Section 3.1 speaks of ReLU   */
/* activations for the layers, and the appendix's network listing for       */
/* time-varying data ends in one).                                          */
/* ------------------------------------------------------------------------ */

/* Forward for one sample; keeps pre-activations z[layer][width] if asked and
 * the output neuron's input in *z_out if asked. */
static double orc_mlp_one_z(const orc_model* m, const double* W, const double* e, double* z_keep, double* z_out)
{
    double a[1024], b[1024];
    const double* in = e;
    int n_in = m->n_in;
    for (int li = 0; li < m->n_layers; ++li) {
        const double* Wl = W + m->w_off[li];
        int no = m->w_out[li];
        for (int o = 0; o < no; ++o) {
            double s = 0.0;
            for (int k = 0; k < n_in; ++k) s += Wl[(int64_t)o * n_in + k] * in[k];
            if (li == m->n_layers - 1) {
                if (z_out) *z_out = s;
                return (m->out_relu && !(s > 0.0)) ? 0.0 : s;
            }
            if (z_keep) z_keep[li * m->width + o] = s;
            b[o] = s > 0.0 ? s : 0.0;
        }
        memcpy(a, b, sizeof(double) * (size_t)no);
        in = a;
        n_in = no;
    }
    return 0.0; /* not reached */
}

static double orc_mlp_one(const orc_model* m, const double* W, const double* e, double* z_keep)
{
    return orc_mlp_one_z(m, W, e, z_keep, NULL);
}

int orc_mlp_fwd(const int32_t* desc, const double* W, const double* feat, int64_t n, double* out)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_mlp_one(&m, W, feat + i * m.n_in, NULL);
    return 0;
}

/* out[n] = Phi(xyz) = MLP(encode(xyz)). */
int orc_forward(const int32_t* desc, const double* params, const float* xyz, int64_t n, double* out)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
    const double* W = params + m.n_table;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double e[1024];
        orc_encode_one(&m, params, xyz + 3 * i, e);
        out[i] = orc_mlp_one(&m, W, e, NULL);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampling step (Section 4).                                               */
/* ------------------------------------------------------------------------ */

/*
 * Cell-centred trilinear sample with clamp-to-edge of a volume with dims
 * (Dx, Dy, Dz), x fastest.  Voxel i has its centre at (i + 1/2)/D, so the
 * sample is exact at voxel centres.
 */
static double orc_volume_at(const float* vol, const int32_t* dims, const float* xyz)
{
    int64_t i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        int64_t D = dims[a];
        double u = (double)xyz[a] * (double)D - 0.5;
        double fl = floor(u);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(D - 2)) fl = (double)(D - 2);
        double tt = u - fl;
        if (tt < 0.0) tt = 0.0;
        if (tt > 1.0) tt = 1.0;
        i0[a] = (int64_t)fl;
        t[a] = tt;
    }
    double s = 0.0;
    for (int k = 0; k < 8; ++k) {
        int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
        int64_t id = (i0[0] + dx) + (int64_t)dims[0] * ((i0[1] + dy) + (int64_t)dims[1] * (i0[2] + dz));
        s += w * (double)vol[id];
    }
    return s;
}

int orc_sample_volume(const float* vol, const int32_t* dims, const float* xyz, int64_t n, double* y)
{
    if (dims[0] < 2 || dims[1] < 2 || dims[2] < 2) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = orc_volume_at(vol, dims, xyz + 3 * i);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Out-of-core sampling (Section 4.1).                                       */
/*                                                                          */
/* Reading: the volume is cut into blocks of b^3 voxels (the last block of   */
/* an axis may be partial), numbered z-major over the block grid             */
/* G_a = ceil(D_a / b).  A buffer of R slots holds blocks.  Block loads are  */
/* numbered j = 0, 1, ...: load j brings block                               */
/* ((r_j >> 40) * n_blocks) >> 24, r_j = SplitMix64(seed, stream 9, j);      */
/* loads 0..R-1 fill slots 0..R-1 before the first sampling step (the warm-  */
/* up), and the refresh before step k >= 1 makes loads                       */
/* j = R + (k-1) S + i, i < S, into slots ((k-1) S + i) mod R (the S oldest). */
/* Sample i of step k takes draws d = 0..6 of stream 10 at index             */
/* (k B + i) 8 + d: the slot ((r_0 >> 40) R) >> 24; a voxel of the slot's    */
/* block, per axis origin_a + (((r_a >> 40) n_a) >> 24) with n_a the block's */
/* extent min(b, D_a - origin_a); the jitter u_a = (r >> 40) 2^-24 from      */
/* d = 4..6.  The coordinate is x_a = (v_a + u_a) / D_a in binary32 (the     */
/* voxel centre moved by U[-1/2, 1/2)), the target the volume's trilinear    */
/* sample at x (orc_volume_at): a one-voxel ghost layer around a block holds */
/* every voxel that sample needs.                                            */
/* ------------------------------------------------------------------------ */
static int64_t orc_ooc_pick(uint64_t r, int64_t n) { return (int64_t)(((r >> 40) * (uint64_t)n) >> 24); }

/* block in every slot after the loads up to and including step `step`'s */
int orc_ooc_slots(const int32_t* dims, int b, int64_t R, int64_t S, uint64_t seed, int64_t step, int64_t* slot_block)
{
    if (b < 1 || R < 1 || S < 1 || S > R || step < 0) return -1;
    int64_t G[3];
    for (int a = 0; a < 3; ++a) G[a] = (dims[a] + b - 1) / b;
    const int64_t nb = G[0] * G[1] * G[2];
    for (int64_t j = 0; j < R; ++j) slot_block[j] = orc_ooc_pick(orc_rng_u64(seed, 9u, (uint64_t)j), nb);
    for (int64_t k = 1; k <= step; ++k)
        for (int64_t i = 0; i < S; ++i) {
            const int64_t j = R + (k - 1) * S + i;
            slot_block[((k - 1) * S + i) % R] = orc_ooc_pick(orc_rng_u64(seed, 9u, (uint64_t)j), nb);
        }
    return 0;
}

/* the B samples of step `step`: coordinates, targets and the block each
 * came from */
int orc_ooc_sample(const float* vol, const int32_t* dims, int b, int64_t R, int64_t S, uint64_t seed, int64_t step,
                   int64_t B, float* xyz, double* y, int64_t* block_of)
{
    int64_t* slots = (int64_t*)malloc(sizeof(int64_t) * (size_t)R);
    if (!slots) return -2;
    if (orc_ooc_slots(dims, b, R, S, seed, step, slots)) {
        free(slots);
        return -1;
    }
    int64_t G[3];
    for (int a = 0; a < 3; ++a) G[a] = (dims[a] + b - 1) / b;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < B; ++i) {
        const uint64_t base = (uint64_t)(step * B + i) * 8u;
        const int64_t blk = slots[orc_ooc_pick(orc_rng_u64(seed, 10u, base), R)];
        const int64_t bc[3] = {blk % G[0], (blk / G[0]) % G[1], blk / (G[0] * G[1])};
        for (int a = 0; a < 3; ++a) {
            const int64_t origin = bc[a] * b;
            const int64_t ext = dims[a] - origin < b ? dims[a] - origin : b;
            const int64_t v = origin + orc_ooc_pick(orc_rng_u64(seed, 10u, base + 1u + (uint64_t)a), ext);
            const float u = (float)(orc_rng_u64(seed, 10u, base + 4u + (uint64_t)a) >> 40) * 0x1p-24f;
            xyz[3 * i + a] = ((float)v + u) / (float)dims[a];
        }
        y[i] = orc_volume_at(vol, dims, xyz + 3 * i);
        if (block_of) block_of[i] = blk;
    }
    free(slots);
    return 0;
}

/* Training batch of step `step`: stream 3, index = step*B*3 + i*3 + axis. */
int orc_batch_coords(uint64_t seed, int64_t step, int64_t B, float* xyz)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < B; ++i)
        for (int a = 0; a < 3; ++a)
            xyz[3 * i + a] = (float)orc_rng_u01(seed, 3u, (uint64_t)(step * B * 3 + i * 3 + a));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Loss and analytic gradient.                                              */
/* kind 0 (L2): L = (1/B) sum_i (Phi(x_i) - y_i)^2;                         */
/* kind 1 (L1, the paper's default loss, Section 3.1):                      */
/*   L = (1/B) sum_i |Phi(x_i) - y_i|, dL/dPhi_i = sign(Phi_i - y_i)/B with  */
/*   sign(0) = 0;                                                           */
/* grad = dL/dparams (all parameters).                                      */
/* ------------------------------------------------------------------------ */
int orc_loss_grad_kind(const int32_t* desc, const double* params, const float* xyz, const double* y, int64_t n,
                       int kind, double* grad, double* loss_out)
{
    if (kind != 0 && kind != 1) return -1;
    orc_model m;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024 || m.n_layers > 16) return -1;
    const double* W = params + m.n_table;
    memset(grad, 0, sizeof(double) * (size_t)m.n_params);
    double* gW = grad + m.n_table;
    /* per-sample feature gradient, then a sequential scatter in sample order */
    double* de_all = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)m.n_in);
    if (!de_all) return -2;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double* gW_t = (double*)calloc((size_t)nt * (size_t)m.n_mlp, sizeof(double));
    double* loss_t = (double*)calloc((size_t)nt, sizeof(double));
    if (!gW_t || !loss_t) {
        free(de_all);
        free(gW_t);
        free(loss_t);
        return -2;
    }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* gw = gW_t + (size_t)tid * (size_t)m.n_mlp;
        double* e = (double*)malloc(sizeof(double) * 1024);
        double* z = (double*)malloc(sizeof(double) * 16 * 1024);
        double* h = (double*)malloc(sizeof(double) * 16 * 1024);
        double* dz = (double*)malloc(sizeof(double) * 1024);
        double* dh = (double*)malloc(sizeof(double) * 1024);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            orc_encode_one(&m, params, xyz + 3 * i, e);
            double zo = 0.0;
            double yhat = orc_mlp_one_z(&m, W, e, z, &zo);
            double r = yhat - y[i];
            double g; /* dL/dz_out: dL/dyhat, times ReLU'(z_out) (0 at 0) with an output ReLU */
            if (kind == 1) {
                loss_t[tid] += fabs(r);
                g = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) / (double)n;
            } else {
                loss_t[tid] += r * r;
                g = 2.0 * r / (double)n;
            }
            if (m.out_relu && !(zo > 0.0)) g = 0.0;
            /* hidden activations h_j = relu(z_j) */
            for (int li = 0; li < m.n_hidden; ++li)
                for (int o = 0; o < m.width; ++o) {
                    double v = z[li * m.width + o];
                    h[li * m.width + o] = v > 0.0 ? v : 0.0;
                }
            /* output layer: yhat = w_out . h_last */
            int last = m.n_layers - 1;
            const double* Wo = W + m.w_off[last];
            for (int k = 0; k < m.width; ++k) {
                gw[m.w_off[last] + k] += g * h[(m.n_hidden - 1) * m.width + k];
                dh[k] = g * Wo[k];
            }
            /* hidden layers, last to first */
            for (int li = m.n_hidden - 1; li >= 0; --li) {
                int nin = m.w_in[li];
                const double* Wl = W + m.w_off[li];
                const double* a_in = (li == 0) ? e : h + (li - 1) * m.width;
                for (int o = 0; o < m.width; ++o) dz[o] = z[li * m.width + o] > 0.0 ? dh[o] : 0.0;
                for (int o = 0; o < m.width; ++o)
                    for (int k = 0; k < nin; ++k) gw[m.w_off[li] + (int64_t)o * nin + k] += dz[o] * a_in[k];
                double* dprev = (li == 0) ? de_all + i * m.n_in : dh;
                double tmp[1024];
                for (int k = 0; k < nin; ++k) {
                    double s = 0.0;
                    for (int o = 0; o < m.width; ++o) s += Wl[(int64_t)o * nin + k] * dz[o];
                    tmp[k] = s;
                }
                memcpy(dprev, tmp, sizeof(double) * (size_t)nin);
            }
        }
        free(e);
        free(z);
        free(h);
        free(dz);
        free(dh);
    }
    double loss = 0.0;
    for (int t = 0; t < nt; ++t) {
        loss += loss_t[t];
        for (int64_t k = 0; k < m.n_mlp; ++k) gW[k] += gW_t[(size_t)t * (size_t)m.n_mlp + (size_t)k];
    }
    /* table gradient: grad[idx][f] += w * de[l*F+f] */
    for (int64_t i = 0; i < n; ++i) {
        const float* p = xyz + 3 * i;
        double x[3] = {orc_clamp01f(p[0]), orc_clamp01f(p[1]), orc_clamp01f(p[2])};
        for (int l = 0; l < m.L; ++l) {
            int64_t idx[8];
            double wt[8];
            orc_corners(&m, l, x, idx, wt);
            for (int k = 0; k < 8; ++k)
                for (int f = 0; f < m.F; ++f) grad[idx[k] * m.F + f] += wt[k] * de_all[i * m.n_in + l * m.F + f];
        }
    }
    if (loss_out) *loss_out = (n > 0) ? loss / (double)n : 0.0;
    free(de_all);
    free(gW_t);
    free(loss_t);
    return 0;
}

int orc_loss_grad(const int32_t* desc, const double* params, const float* xyz, const double* y, int64_t n,
                  double* grad, double* loss_out)
{
    return orc_loss_grad_kind(desc, params, xyz, y, n, 0, grad, loss_out);
}

/* ------------------------------------------------------------------------ */
/* Exponentially decaying learning rate (Section 3.1; decay start, interval */
/* and base from the appendix's default optimiser).  Reading: the rate is    */
/* constant for the first `start` steps and is then multiplied by `base`     */
/* once every `interval` steps: step k (0-based) uses                        */
/* lr * base^floor((k - start) / interval) for k >= start.  interval <= 0    */
/* means no decay.                                                          */
/* ------------------------------------------------------------------------ */
double orc_lr_at(double lr, int64_t k, int64_t start, int64_t interval, double base)
{
    if (interval <= 0 || k < start) return lr;
    int64_t n = (k - start) / interval;
    double f = 1.0;
    for (int64_t i = 0; i < n; ++i) f *= base;
    return lr * f;
}

/* ------------------------------------------------------------------------ */
/* Adam (Kingma and Ba 2014), dense, bias-corrected, eps outside the root.  */
/* t is the 1-based step number.  L2 regularisation (appendix default       */
/* optimiser, read as a penalty (l2_reg/2)|w|^2 on the network weights):     */
/* l2_reg * theta_i joins the gradient of every index i >= reg_from.         */
/* ------------------------------------------------------------------------ */
int orc_adam_reg(int64_t n, int64_t reg_from, double* theta, double* m, double* v, const double* g, int64_t t,
                 double lr, double b1, double b2, double eps, double l2_reg)
{
    double c1 = 1.0 - pow(b1, (double)t);
    double c2 = 1.0 - pow(b2, (double)t);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double gi = g[i] + (i >= reg_from ? l2_reg * theta[i] : 0.0);
        m[i] = b1 * m[i] + (1.0 - b1) * gi;
        v[i] = b2 * v[i] + (1.0 - b2) * gi * gi;
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}

int orc_adam(int64_t n, double* theta, double* m, double* v, const double* g, int64_t t, double lr, double b1,
             double b2, double eps)
{
    return orc_adam_reg(n, n, theta, m, v, g, t, lr, b1, b2, eps, 0.0);
}

/*
 * `steps` training steps of batch B on a volume: coordinates of step s from
 * orc_batch_coords(seed, step0 + s), targets by orc_sample_volume, loss of
 * `kind` (0 L2, 1 L1), Adam at 1-based step t = step0 + s + 1 with the rate
 * orc_lr_at(lr, t - 1, ...) and L2 regularisation of the MLP weights.
 * opt = {lr, beta1, beta2, eps, l2_reg, decay_start, decay_interval,
 * decay_base}.  m and v are caller-owned state.
 */
int orc_train_opt(const int32_t* desc, double* params, double* adam_m, double* adam_v, const float* vol,
                  const int32_t* dims, uint64_t seed, int64_t step0, int64_t steps, int64_t B, int kind,
                  const double* opt, double* losses)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m)) return -1;
    float* xyz = (float*)malloc(sizeof(float) * 3 * (size_t)B);
    double* y = (double*)malloc(sizeof(double) * (size_t)B);
    double* g = (double*)malloc(sizeof(double) * (size_t)m.n_params);
    if (!xyz || !y || !g) {
        free(xyz);
        free(y);
        free(g);
        return -2;
    }
    int rc = 0;
    for (int64_t s = 0; s < steps && rc == 0; ++s) {
        const int64_t k = step0 + s;
        orc_batch_coords(seed, k, B, xyz);
        orc_sample_volume(vol, dims, xyz, B, y);
        double loss = 0.0;
        rc = orc_loss_grad_kind(desc, params, xyz, y, B, kind, g, &loss);
        if (losses) losses[s] = loss;
        if (rc == 0) {
            double lr = orc_lr_at(opt[0], k, (int64_t)opt[5], (int64_t)opt[6], opt[7]);
            orc_adam_reg(m.n_params, m.n_table, params, adam_m, adam_v, g, k + 1, lr, opt[1], opt[2], opt[3], opt[4]);
        }
    }
    free(xyz);
    free(y);
    free(g);
    return rc;
}

int orc_train(const int32_t* desc, double* params, double* adam_m, double* adam_v, const float* vol,
              const int32_t* dims, uint64_t seed, int64_t step0, int64_t steps, int64_t B, double lr, double b1,
              double b2, double eps, double* losses)
{
    const double opt[8] = {lr, b1, b2, eps, 0.0, 0.0, 0.0, 1.0};
    return orc_train_opt(desc, params, adam_m, adam_v, vol, dims, seed, step0, steps, B, 0, opt, losses);
}

/* ------------------------------------------------------------------------ */
/* Decode and PSNR (Section 6): MSE over all voxel centres (i+1/2)/D.        */
/* ------------------------------------------------------------------------ */
int orc_mse_grid(const int32_t* desc, const double* params, const float* vol, const int32_t* dims, double* mse)
{
    orc_model m;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
    const double* W = params + m.n_table;
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
    for (int64_t z = 0; z < nz; ++z) {
        double e[1024];
        for (int64_t yv = 0; yv < ny; ++yv)
            for (int64_t xv = 0; xv < nx; ++xv) {
                float p[3] = {((float)xv + 0.5f) / (float)nx, ((float)yv + 0.5f) / (float)ny,
                              ((float)z + 0.5f) / (float)nz};
                orc_encode_one(&m, params, p, e);
                double d = orc_mlp_one(&m, W, e, NULL) - (double)vol[xv + nx * (yv + ny * z)];
                acc += d * d;
            }
    }
    *mse = acc / (double)(nx * ny * nz);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Ray-marched emission-absorption rendering (Section 5.2.1).               */
/*                                                                          */
/* Ray geometry is binary32, one rounding per operation, no FMA:            */
/*   dir = (W + (px+1/2) U) + (py+1/2) V, d = dir / sqrt(dir.dir);          */
/*   slab test against [0,1]^3 with inv = 1/d; t_near = max(t_min, 0);       */
/*   hit iff t_near < t_max; n = max(0, ceil((t_max - t_near)/dt - j));      */
/*   t_k = t_near + (k + j) dt; p_k = o + t_k d.                             */
/* Everything after p_k is FP64: Phi(p_k) -> v = clamp(Phi, 0, 1) ->         */
/* linear lookup in a 256-entry RGBA table -> front-to-back compositing,     */
/* stopping after the sample at which accumulated alpha reaches 0.99.        */
/* cam = { o[3], U[3], V[3], W[3] }.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    float o[3], d[3], t0, j;
    uint32_t n;
} orc_ray;

static orc_ray orc_make_ray(const float* cam, int W, int px, int py, uint32_t frame_seed, float dt)
{
    orc_ray r;
    float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float dir[3];
    for (int a = 0; a < 3; ++a) {
        float t1 = fx * cam[3 + a];
        float t2 = cam[9 + a] + t1;
        float t3 = fy * cam[6 + a];
        dir[a] = t2 + t3;
    }
    float q0 = dir[0] * dir[0], q1 = dir[1] * dir[1], q2 = dir[2] * dir[2];
    float n2 = (q0 + q1) + q2;
    float nrm = sqrtf(n2);
    float tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        r.o[a] = cam[a];
        r.d[a] = dir[a] / nrm;
        float inv = 1.0f / r.d[a];
        float ta = (0.0f - r.o[a]) * inv;
        float tb = (1.0f - r.o[a]) * inv;
        tmin = fmaxf(tmin, fminf(ta, tb));
        tmax = fminf(tmax, fmaxf(ta, tb));
    }
    float tn = fmaxf(tmin, 0.0f);
    r.t0 = tn;
    r.j = (float)orc_rng_u01((uint64_t)frame_seed, 5u, (uint64_t)py * (uint64_t)W + (uint64_t)px);
    r.n = 0;
    if (tn < tmax) {
        float span = tmax - tn;
        float q = span / dt;
        /* a chord of the unit cube is at most sqrt(3) long: a ray with more
         * than 2^24 steps (or a NaN span) is degenerate and gets no samples */
        if (q <= 16777216.0f) {
            float c = ceilf(q - r.j);
            if (c > 0.0f) r.n = (uint32_t)c;
        }
    }
    return r;
}

static void orc_ray_point(const orc_ray* r, uint32_t k, float dt, float p[3])
{
    float kj = (float)k + r->j;
    float t = r->t0 + kj * dt;
    for (int a = 0; a < 3; ++a) {
        float td = t * r->d[a];
        p[a] = r->o[a] + td;
    }
}

/* Per-pixel geometric sample counts n[H*W] and the k-th sample coordinate
 * of pixel `pix` (for bit-exact coordinate checks). */
int orc_ray_counts(const float* cam, int W, int H, uint32_t frame_seed, float dt, uint32_t* n)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)W * H; ++p) {
        orc_ray r = orc_make_ray(cam, W, (int)(p % W), (int)(p / W), frame_seed, dt);
        n[p] = r.n;
    }
    return 0;
}

int orc_ray_points(const float* cam, int W, int H, uint32_t frame_seed, float dt, int64_t pix, uint32_t k0,
                   uint32_t count, float* xyz)
{
    (void)H;
    orc_ray r = orc_make_ray(cam, W, (int)(pix % W), (int)(pix / W), frame_seed, dt);
    for (uint32_t k = 0; k < count; ++k) orc_ray_point(&r, k0 + k, dt, xyz + 3 * k);
    return 0;
}

/*
 * Render the pixels listed in pix[n_pix] (row-major pixel ids, py*W + px).
 * rgba[n_pix][4] (premultiplied colour, accumulated alpha), n_geo[n_pix]
 * (geometric count), n_used[n_pix] (samples composited before stopping).
 */
/* ------------------------------------------------------------------------ */
/* Macro-cells (Section 5.3): disjoint cells of `cell` voxels per axis over  */
/* a D_x x D_y x D_z volume, M_a = ceil(D_a / cell) per axis (the grid may   */
/* extend past the volume).  Reading: a point p (clamped to [0,1], NaN as 0) */
/* lies in voxel floor(p_a D_a), the product rounded to binary32, and in     */
/* cell min(voxel / cell, M_a - 1).  Each cell keeps the range of the        */
/* values seen in it; per the online construction of Section 5.3 the values  */
/* are the training samples' targets.  The maximum opacity mu of a cell is    */
/* the largest alpha the transfer function takes over its range, 0 for a     */
/* cell no sample has reached.                                               */
/* ------------------------------------------------------------------------ */
static int64_t orc_mc_index(const float p[3], const int32_t* dims, int cell)
{
    int64_t c[3], M[3];
    for (int a = 0; a < 3; ++a) {
        M[a] = (dims[a] + cell - 1) / cell;
        float q = (float)orc_clamp01f(p[a]);
        float s = q * (float)dims[a];
        int64_t vox = (int64_t)floorf(s);
        c[a] = vox / cell;
        if (c[a] > M[a] - 1) c[a] = M[a] - 1;
    }
    return (c[2] * M[1] + c[1]) * M[0] + c[0];
}

int orc_mc_cells(const int32_t* dims, int cell, const float* xyz, int64_t n, int64_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_mc_index(xyz + 3 * i, dims, cell);
    return 0;
}

/* vmin/vmax of every cell over the samples, in sample order; cells start
 * empty (vmin = +inf, vmax = -inf) unless the caller passes earlier ranges. */
int orc_mc_update(const int32_t* dims, int cell, const float* xyz, const float* values, int64_t n, double* vmin,
                  double* vmax)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = orc_mc_index(xyz + 3 * i, dims, cell);
        double v = values[i];
        if (v < vmin[c]) vmin[c] = v;
        if (v > vmax[c]) vmax[c] = v;
    }
    return 0;
}

/* alpha of the shading transfer function at v: u = 255 clamp(v, 0, 1) and
 * its fraction in binary32 (as the shading forms them), the blend in FP64 */
static double orc_tf_alpha(const float* lut, float v)
{
    float c = v > 0.0f ? (v < 1.0f ? v : 1.0f) : 0.0f;
    float u = 255.0f * c;
    float fi = floorf(u);
    if (fi > 254.0f) fi = 254.0f;
    int i0 = (int)fi;
    float fr = u - fi;
    return (double)lut[4 * i0 + 3] + (double)fr * ((double)lut[4 * (i0 + 1) + 3] - (double)lut[4 * i0 + 3]);
}

/* mu = max of the piecewise-linear alpha over [vmin, vmax]: the two ends and
 * every node strictly inside */
int orc_mc_opacity(const double* vmin, const double* vmax, int64_t n_cells, const float* lut, double* mu)
{
    for (int64_t c = 0; c < n_cells; ++c) {
        if (!(vmin[c] <= vmax[c])) {
            mu[c] = 0.0;
            continue;
        }
        float lo = (float)vmin[c], hi = (float)vmax[c];
        double m = orc_tf_alpha(lut, lo);
        double b = orc_tf_alpha(lut, hi);
        if (b > m) m = b;
        float ul = 255.0f * (lo > 0.0f ? (lo < 1.0f ? lo : 1.0f) : 0.0f);
        float uh = 255.0f * (hi > 0.0f ? (hi < 1.0f ? hi : 1.0f) : 0.0f);
        for (int i = 0; i < 256; ++i)
            if ((float)i > ul && (float)i < uh && (double)lut[4 * i + 3] > m) m = lut[4 * i + 3];
        mu[c] = m;
    }
    return 0;
}

/*
 * Rendering of the listed pixels; with mu != NULL a sample whose macro-cell
 * has mu = 0 is skipped (not evaluated, not composited): empty-space
 * skipping.  n_used counts composited samples up to termination.
 */
int orc_render_pixels_mc(const int32_t* desc, const double* params, const float* cam, const float* lut, int W,
                         int H, float dt, uint32_t frame_seed, const int64_t* pix, int64_t n_pix,
                         const int32_t* mc_dims, int mc_cell, const double* mu, double* rgba, uint32_t* n_geo,
                         uint32_t* n_used)
{
    orc_model m;
    (void)H;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
    const double* Wm = params + m.n_table;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t p = pix[q];
        orc_ray r = orc_make_ray(cam, W, (int)(p % W), (int)(p / W), frame_seed, dt);
        double C[3] = {0.0, 0.0, 0.0}, A = 0.0;
        uint32_t used = 0;
        double e[1024];
        for (uint32_t k = 0; k < r.n; ++k) {
            float pt[3];
            orc_ray_point(&r, k, dt, pt);
            if (mu && !(mu[orc_mc_index(pt, mc_dims, mc_cell)] > 0.0)) continue;
            orc_encode_one(&m, params, pt, e);
            double v = orc_mlp_one(&m, Wm, e, NULL);
            if (!(v > 0.0)) v = 0.0;
            if (v > 1.0) v = 1.0;
            double u = 255.0 * v;
            double fi = floor(u);
            if (fi > 254.0) fi = 254.0;
            int i0 = (int)fi;
            double f = u - fi;
            double c4[4];
            for (int ch = 0; ch < 4; ++ch)
                c4[ch] = (double)lut[4 * i0 + ch] * (1.0 - f) + (double)lut[4 * (i0 + 1) + ch] * f;
            double a = c4[3];
            for (int ch = 0; ch < 3; ++ch) C[ch] += (1.0 - A) * a * c4[ch];
            A += (1.0 - A) * a;
            used += 1;
            if (A >= 0.99) break;
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = C[ch];
        rgba[4 * q + 3] = A;
        n_geo[q] = r.n;
        n_used[q] = used;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adaptive ray marching through macro-cells (Section 5.3).                  */
/*                                                                          */
/* Reading: samples stay on the ray's grid t_k = t_near + (k + j) dt.  From  */
/* sample k in cell c (the cell of its binary32 point):                      */
/*   - mu(c) = 0: the cell is transparent and bypassed: k moves to the first */
/*     sample outside c;                                                    */
/*   - otherwise the sample is evaluated and represents m grid steps, where  */
/*     m = min(n(mu), exit(c) - k, n_r - k), n(mu) = max(1, floor(sbar)) and */
/*     sbar = max(s1 + (s2 - s1) |min(mu,1) - 1|^p, s1) with s1 = 1 grid     */
/*     step (binary32, one rounding per operation, the power by repeated     */
/*     multiplication, p a positive integer); its opacity is corrected to    */
/*     1 - (1 - alpha)^m (alpha itself when m = 1), and k moves by m.        */
/* exit(c), the first sample outside c, is found by a DDA step: the ray's    */
/* exit from the cell's box, the grid index just past it, and an exact       */
/* correction by testing the cells of the neighbouring samples.              */
/* ------------------------------------------------------------------------ */
int orc_adaptive_steps(float mu, float s2, int p)
{
    float m = mu < 1.0f ? mu : 1.0f;
    float d = fabsf(m - 1.0f);
    float pw = 1.0f;
    for (int i = 0; i < p; ++i) pw = pw * d;
    float t = (s2 - 1.0f) * pw;
    float sb = 1.0f + t;
    if (sb < 1.0f) sb = 1.0f;
    return (int)floorf(sb);
}

static int64_t orc_ray_cell(const orc_ray* r, uint32_t k, float dt, const int32_t* dims, int cell)
{
    float pt[3];
    orc_ray_point(r, k, dt, pt);
    return orc_mc_index(pt, dims, cell);
}

/* first sample index > k outside the cell of sample k, by scanning */
static uint32_t orc_cell_exit_scan(const orc_ray* r, uint32_t k, float dt, const int32_t* dims, int cell)
{
    int64_t c = orc_ray_cell(r, k, dt, dims, cell);
    uint32_t q = k + 1;
    while (q < r->n && orc_ray_cell(r, q, dt, dims, cell) == c) ++q;
    return q;
}

/* the same by a DDA step: leave the cell's box along the ray, take the grid
 * index past that parameter, and correct it on the samples' own cells */
static uint32_t orc_cell_exit_dda(const orc_ray* r, uint32_t k, float dt, const int32_t* dims, int cell)
{
    float pt[3];
    orc_ray_point(r, k, dt, pt);
    int64_t c = orc_mc_index(pt, dims, cell);
    float t_exit = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (r->d[a] == 0.0f) continue;
        int64_t M = (dims[a] + cell - 1) / cell;
        float q = (float)orc_clamp01f(pt[a]);
        int64_t ca = (int64_t)floorf(q * (float)dims[a]) / cell;
        if (ca > M - 1) ca = M - 1;
        float bound;
        if (r->d[a] > 0.0f) {
            if (ca == M - 1) continue; /* the last cell reaches the cube's face */
            bound = (float)((ca + 1) * cell) / (float)dims[a];
        } else {
            if (ca == 0) continue;
            bound = (float)(ca * cell) / (float)dims[a];
        }
        float ta = (bound - r->o[a]) / r->d[a];
        if (ta < t_exit) t_exit = ta;
    }
    uint32_t q;
    if (!(t_exit < INFINITY)) {
        q = r->n;
    } else {
        float g = ceilf((t_exit - r->t0) / dt - r->j);
        q = g <= (float)(k + 1) ? k + 1 : (g >= (float)r->n ? r->n : (uint32_t)g);
    }
    while (q < r->n && orc_ray_cell(r, q, dt, dims, cell) == c) ++q;
    while (q > k + 1 && orc_ray_cell(r, q - 1, dt, dims, cell) != c) --q;
    return q;
}

/* the cells a pixel's ray visits and the first sample in each: by the DDA
 * step (mode 1) or by scanning every sample (mode 0) */
int orc_mc_traverse(const float* cam, int W, uint32_t frame_seed, float dt, int64_t pix, const int32_t* dims,
                    int cell, int mode, int64_t* cells, uint32_t* first, int64_t cap, int64_t* count)
{
    orc_ray r = orc_make_ray(cam, W, (int)(pix % W), (int)(pix / W), frame_seed, dt);
    int64_t n = 0;
    uint32_t k = 0;
    while (k < r.n) {
        if (n >= cap) return -2;
        cells[n] = orc_ray_cell(&r, k, dt, dims, cell);
        first[n] = k;
        ++n;
        k = mode ? orc_cell_exit_dda(&r, k, dt, dims, cell) : orc_cell_exit_scan(&r, k, dt, dims, cell);
    }
    *count = n;
    return 0;
}

/*
 * Adaptive ray marching of the listed pixels through macro-cells of maximum
 * opacity mu (binary32 values, as the renderer stores them): s2 the largest
 * step in grid steps, p the exponent.  Outputs as orc_render_pixels; n_used
 * counts evaluated samples up to termination.
 */
int orc_render_pixels_adaptive(const int32_t* desc, const double* params, const float* cam, const float* lut, int W,
                               int H, float dt, uint32_t frame_seed, const int64_t* pix, int64_t n_pix,
                               const int32_t* mc_dims, int mc_cell, const float* mu, float s2, int p, double* rgba,
                               uint32_t* n_geo, uint32_t* n_used)
{
    orc_model m;
    (void)H;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024 || p < 1 || p > 8 || !(s2 >= 1.0f))
        return -1;
    const double* Wm = params + m.n_table;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t px = pix[q];
        orc_ray r = orc_make_ray(cam, W, (int)(px % W), (int)(px / W), frame_seed, dt);
        double C[3] = {0.0, 0.0, 0.0}, A = 0.0;
        uint32_t used = 0;
        double e[1024];
        uint32_t k = 0;
        while (k < r.n) {
            float pt[3];
            orc_ray_point(&r, k, dt, pt);
            float muc = mu[orc_mc_index(pt, mc_dims, mc_cell)];
            if (!(muc > 0.0f)) {
                k = orc_cell_exit_dda(&r, k, dt, mc_dims, mc_cell);
                continue;
            }
            uint32_t steps = (uint32_t)orc_adaptive_steps(muc, s2, p);
            uint32_t kn = k + 1;
            if (steps > 1) {
                uint32_t ke = orc_cell_exit_dda(&r, k, dt, mc_dims, mc_cell);
                kn = k + steps < ke ? k + steps : ke;
            }
            if (kn > r.n) kn = r.n;
            uint32_t span = kn - k;
            orc_encode_one(&m, params, pt, e);
            double v = orc_mlp_one(&m, Wm, e, NULL);
            if (!(v > 0.0)) v = 0.0;
            if (v > 1.0) v = 1.0;
            double u = 255.0 * v;
            double fi = floor(u);
            if (fi > 254.0) fi = 254.0;
            int i0 = (int)fi;
            double f = u - fi;
            double c4[4];
            for (int ch = 0; ch < 4; ++ch)
                c4[ch] = (double)lut[4 * i0 + ch] * (1.0 - f) + (double)lut[4 * (i0 + 1) + ch] * f;
            double a = c4[3];
            if (span > 1) a = 1.0 - pow(1.0 - a, (double)span); /* opacity of `span` grid steps */
            for (int ch = 0; ch < 3; ++ch) C[ch] += (1.0 - A) * a * c4[ch];
            A += (1.0 - A) * a;
            used += 1;
            if (A >= 0.99) break;
            k = kn;
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = C[ch];
        rgba[4 * q + 3] = A;
        n_geo[q] = r.n;
        n_used[q] = used;
    }
    return 0;
}

int orc_render_pixels(const int32_t* desc, const double* params, const float* cam, const float* lut, int W, int H,
                      float dt, uint32_t frame_seed, const int64_t* pix, int64_t n_pix, double* rgba,
                      uint32_t* n_geo, uint32_t* n_used)
{
    return orc_render_pixels_mc(desc, params, cam, lut, W, H, dt, frame_seed, pix, n_pix, NULL, 1, NULL, rgba,
                                n_geo, n_used);
}

/* ------------------------------------------------------------------------ */
/* Shared pieces of the shadow ray marcher and the path tracer.              */
/* ------------------------------------------------------------------------ */

/* v / |v| in binary32, |v| formed as the camera rule forms it */
static void orc_unit3(const float v[3], float out[3])
{
    float q0 = v[0] * v[0], q1 = v[1] * v[1], q2 = v[2] * v[2];
    float nrm = sqrtf((q0 + q1) + q2);
    for (int a = 0; a < 3; ++a) out[a] = v[a] / nrm;
}

/* slab test of o + t d against [0,1]^3 (binary32): t_near = max(t_min, 0) */
static void orc_slab(const float o[3], const float d[3], float* tn, float* tf)
{
    float tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        float inv = 1.0f / d[a];
        float ta = (0.0f - o[a]) * inv;
        float tb = (1.0f - o[a]) * inv;
        tmin = fmaxf(tmin, fminf(ta, tb));
        tmax = fminf(tmax, fmaxf(ta, tb));
    }
    *tn = fmaxf(tmin, 0.0f);
    *tf = tmax;
}

/* Ray from o along the unit direction d with jitter j, sample count by the
 * camera rays' rule: n = max(0, ceil((t_far - t_near)/dt - j)) */
static orc_ray orc_ray_from(const float o[3], const float d[3], float j, float dt)
{
    orc_ray r;
    float tn, tf;
    orc_slab(o, d, &tn, &tf);
    for (int a = 0; a < 3; ++a) {
        r.o[a] = o[a];
        r.d[a] = d[a];
    }
    r.t0 = tn;
    r.j = j;
    r.n = 0;
    if (tn < tf) {
        float q = (tf - tn) / dt;
        if (q <= 16777216.0f) {
            float c = ceilf(q - j);
            if (c > 0.0f) r.n = (uint32_t)c;
        }
    }
    return r;
}

/* transfer function at the network value phi: rgba by the linear blend of
 * the ray marcher (FP64) */
static void orc_tf(const float* lut, double phi, double c4[4])
{
    double v = phi > 0.0 ? (phi < 1.0 ? phi : 1.0) : 0.0;
    double u = 255.0 * v;
    double fi = floor(u);
    if (fi > 254.0) fi = 254.0;
    int i0 = (int)fi;
    double f = u - fi;
    for (int ch = 0; ch < 4; ++ch) c4[ch] = (double)lut[4 * i0 + ch] * (1.0 - f) + (double)lut[4 * (i0 + 1) + ch] * f;
}

/*
 * Ray marching with a single-shot heuristic shadow (Section 5.2; Brownlee et
 * al.: only the point of highest contribution is shaded).
 *
 * Reading: the primary ray is marched and composited as orc_render_pixels_mc
 * (with mu != NULL, samples in cells of mu = 0 skipped).  Its sample of
 * largest contribution w_k = (1 - A_{k-1}) alpha_k (the first one on ties;
 * none when every w_k is 0) is the shading point p*, its binary32 sample
 * position.  A shadow ray leaves p* along the unit light direction l (binary32,
 * l / |l|) with the pixel's jitter j and the primary rays' count rule; its
 * samples t_k = t_near + (k + j) dt for k >= 1 (k = 0, next to p* itself, is
 * left out), with the same skipping, give the transmittance
 * T = prod (1 - alpha_k), ending after the sample at which T <= 0.01.  The
 * pixel is (T C, A): T attenuates the whole primary colour.
 * kstar[q] is the index k of p* (UINT32_MAX when there is none).
 */
int orc_render_pixels_shadow(const int32_t* desc, const double* params, const float* cam, const float* lut, int W,
                             int H, float dt, uint32_t frame_seed, const int64_t* pix, int64_t n_pix,
                             const int32_t* mc_dims, int mc_cell, const double* mu, const float* light, double* rgba,
                             uint32_t* n_geo, uint32_t* n_used, uint32_t* kstar)
{
    orc_model m;
    (void)H;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
    const double* Wm = params + m.n_table;
    float l[3];
    orc_unit3(light, l);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t p = pix[q];
        orc_ray r = orc_make_ray(cam, W, (int)(p % W), (int)(p / W), frame_seed, dt);
        double C[3] = {0.0, 0.0, 0.0}, A = 0.0, wbest = 0.0;
        int64_t best = -1;
        uint32_t used = 0;
        double e[1024], c4[4];
        for (uint32_t k = 0; k < r.n; ++k) {
            float pt[3];
            orc_ray_point(&r, k, dt, pt);
            if (mu && !(mu[orc_mc_index(pt, mc_dims, mc_cell)] > 0.0)) continue;
            orc_encode_one(&m, params, pt, e);
            orc_tf(lut, orc_mlp_one(&m, Wm, e, NULL), c4);
            double w = (1.0 - A) * c4[3];
            if (w > wbest) {
                wbest = w;
                best = k;
            }
            for (int ch = 0; ch < 3; ++ch) C[ch] += w * c4[ch];
            A += w;
            used += 1;
            if (A >= 0.99) break;
        }
        double T = 1.0;
        if (best >= 0) {
            float ps[3];
            orc_ray_point(&r, (uint32_t)best, dt, ps);
            orc_ray s = orc_ray_from(ps, l, r.j, dt);
            for (uint32_t k = 1; k < s.n; ++k) {
                float pt[3];
                orc_ray_point(&s, k, dt, pt);
                if (mu && !(mu[orc_mc_index(pt, mc_dims, mc_cell)] > 0.0)) continue;
                orc_encode_one(&m, params, pt, e);
                orc_tf(lut, orc_mlp_one(&m, Wm, e, NULL), c4);
                T *= 1.0 - c4[3];
                if (T <= 0.01) break;
            }
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = T * C[ch];
        rgba[4 * q + 3] = A;
        n_geo[q] = r.n;
        n_used[q] = used;
        kstar[q] = best >= 0 ? (uint32_t)best : UINT32_MAX;
    }
    return 0;
}

/*
 * Volumetric path tracing with Woodcock tracking (Section 5.2.2, Algorithm 1)
 * and next-event estimation by shadow rays, with macro-cell majorants walked
 * by optical thickness (Section 5.3, Eqs. 1 and 2; Hofmann et al.).
 *
 * Readings (the paper gives the structure, not the estimator):
 *   - medium: extinction sigma(x) = density * alpha(phi(x)) and albedo
 *     rgb(phi(x)), both from the transfer function as the ray marcher reads
 *     it (phi clamped to [0,1], linear blend); the phase function is
 *     isotropic, sampled exactly, so a scattering event multiplies the
 *     throughput by the albedo;
 *   - majorant: density * mu(c) in macro-cell c (mu the cells' opacities, as
 *     binary32); without macro-cells density * max_i alpha_i over the table,
 *     for the whole cube;
 *   - a directional light of radiance E along the unit direction l (binary32,
 *     l / |l|, pointing towards the light) and a background radiance B for
 *     rays that leave the cube;
 *   - the path state machine of the paper's listing: a scattering ray that
 *     meets a real collision becomes a shadow ray from that point towards
 *     the light; a shadow ray that leaves the cube adds beta E / (4 pi) (the
 *     isotropic phase value), one that meets a real collision adds nothing;
 *     either way the path then continues as a scattering ray from the same
 *     point in a new direction; a scattering ray that leaves the cube adds
 *     beta B and ends the path;
 *   - Russian roulette at the real collisions of scattering rays after the
 *     first rr_depth of them: survive with q = min(1, max_c beta_c), then
 *     beta /= q; the path also ends after max_depth such collisions (once
 *     their shadow ray is done) and after 2^16 tentative collisions;
 *   - geometry in binary32 (one rounding per operation): positions
 *     o + t d, distances, optical thickness sums; the transcendental values
 *     (-ln(1 - zeta), cos, sin, sqrt of the direction) in FP64, rounded to
 *     binary32; radiance and throughput in FP64 here;
 *   - random numbers: stream 8 of the counter generator, index
 *     ((pixel * spp + s) * 2^24 + i) for the i-th draw of path s of a pixel,
 *     drawn in this order: zeta for each tracking step, xi at each tentative
 *     collision, the roulette u when it applies, u1 and u2 for each new
 *     direction (z = 1 - 2 u1, phi = 2 pi u2).
 *
 * Tracking from distance t with target thickness tau = -ln(1 - zeta): with
 * macro-cells, the walk starts in the cell of the point at t and visits
 * cells by a 3-D DDA (cell boundaries at multiples of cell/dims, an axis
 * steps when its boundary distance equals the segment's end); the first
 * cell in which the accumulated thickness would exceed tau holds the
 * collision t_c = t_i + (tau - acc) / m_i.  Without macro-cells,
 * t_c = t + tau / m.  Reaching t_far first means the ray leaves the cube.
 * A tentative collision is real when xi * m < density * alpha(phi(x)).
 *
 * Output per pixel: the mean radiance over spp paths (rgb) and the fraction
 * of paths whose camera ray met a real collision (alpha); n_real and n_samp
 * count real and tentative collisions over the pixel's paths.
 */
#define ORC_PT_MAX_SAMPLES 65536u
#define ORC_PI 3.14159265358979323846

typedef struct {
    float density, light[3], E[3], B[3];
    int spp, rr_depth, max_depth;
} orc_pt_opts;

static int orc_track(const float o[3], const float d[3], float t, float tf, float tau, float density, float amax,
                     const int32_t* dims, int cell, const float* mu, float* tc, float* maj)
{
    if (!mu) {
        float m = density * amax;
        if (!(m > 0.0f)) return 0;
        float tt = t + tau / m;
        if (!(tt < tf)) return 0;
        *tc = tt;
        *maj = m;
        return 1;
    }
    int64_t M[3], ca[3];
    for (int a = 0; a < 3; ++a) {
        M[a] = (dims[a] + cell - 1) / cell;
        float pa = o[a] + t * d[a];
        float qa = (float)orc_clamp01f(pa);
        ca[a] = (int64_t)floorf(qa * (float)dims[a]) / cell;
        if (ca[a] > M[a] - 1) ca[a] = M[a] - 1;
    }
    float acc = 0.0f;
    for (int64_t it = 0; it < M[0] + M[1] + M[2] + 3; ++it) {
        float ta[3], tb = tf;
        for (int a = 0; a < 3; ++a) {
            ta[a] = INFINITY;
            if (d[a] > 0.0f) {
                int64_t b = (ca[a] + 1) * cell;
                if (b > dims[a]) b = dims[a];
                ta[a] = ((float)b / (float)dims[a] - o[a]) / d[a];
            } else if (d[a] < 0.0f) {
                ta[a] = ((float)(ca[a] * cell) / (float)dims[a] - o[a]) / d[a];
            }
            tb = fminf(tb, ta[a]);
        }
        float seg = tb - t;
        if (seg < 0.0f) seg = 0.0f;
        float m = density * mu[(ca[2] * M[1] + ca[1]) * M[0] + ca[0]];
        float dtau = m * seg;
        if (m > 0.0f && acc + dtau > tau) {
            *tc = t + (tau - acc) / m;
            *maj = m;
            return 1;
        }
        acc = acc + dtau;
        if (!(tb < tf)) return 0;
        for (int a = 0; a < 3; ++a)
            if (d[a] != 0.0f && ta[a] == tb) {
                ca[a] += d[a] > 0.0f ? 1 : -1;
                if (ca[a] < 0 || ca[a] >= M[a]) return 0;
            }
        t = tb;
    }
    return 0;
}

static void orc_pt_path(const orc_model* m, const double* params, const double* Wm, const float* lut,
                        const orc_pt_opts* po, const float l[3], float amax, const int32_t* dims, int cell,
                        const float* mu, uint64_t seed, uint64_t key, const float eye[3], const float dcam[3],
                        double L[3], int* hit, uint32_t* n_samp, uint32_t* n_real)
{
    uint64_t i = 0;
    double e[1024], c4[4], beta[3] = {1.0, 1.0, 1.0};
    float o[3], d[3], xs[3], t, tf;
    for (int a = 0; a < 3; ++a) {
        o[a] = eye[a];
        d[a] = dcam[a];
    }
    orc_slab(o, d, &t, &tf);
    if (!(t < tf)) {
        for (int ch = 0; ch < 3; ++ch) L[ch] += po->B[ch];
        return;
    }
    int shadow = 0, depth = 0;
    uint32_t samples = 0;
    for (;;) {
        int new_dir = 0;
        if (samples >= ORC_PT_MAX_SAMPLES) return;
        float zeta = (float)orc_rng_u01(seed, 8u, key + i++);
        float tau = (float)(-log(1.0 - (double)zeta));
        float tc, maj;
        if (!orc_track(o, d, t, tf, tau, po->density, amax, dims, cell, mu, &tc, &maj)) {
            if (!shadow) {
                for (int ch = 0; ch < 3; ++ch) L[ch] += beta[ch] * (double)po->B[ch];
                return;
            }
            for (int ch = 0; ch < 3; ++ch) L[ch] += beta[ch] * (double)po->E[ch] / (4.0 * ORC_PI);
            new_dir = 1;
        } else {
            float x[3];
            for (int a = 0; a < 3; ++a) x[a] = o[a] + tc * d[a];
            orc_encode_one(m, params, x, e);
            orc_tf(lut, orc_mlp_one(m, Wm, e, NULL), c4);
            ++samples;
            ++*n_samp;
            float xi = (float)orc_rng_u01(seed, 8u, key + i++);
            if (!((double)xi * (double)maj < (double)po->density * c4[3])) {
                t = tc; /* null collision: the ray goes on */
                continue;
            }
            ++*n_real;
            if (shadow) {
                new_dir = 1; /* the light is blocked */
            } else {
                if (depth == 0) *hit = 1;
                ++depth;
                if (depth > po->rr_depth) {
                    double q = beta[0];
                    if (beta[1] > q) q = beta[1];
                    if (beta[2] > q) q = beta[2];
                    if (q > 1.0) q = 1.0;
                    double u = orc_rng_u01(seed, 8u, key + i++);
                    if (u >= q) return;
                    for (int ch = 0; ch < 3; ++ch) beta[ch] /= q;
                }
                for (int ch = 0; ch < 3; ++ch) beta[ch] *= c4[ch];
                for (int a = 0; a < 3; ++a) {
                    xs[a] = x[a];
                    o[a] = x[a];
                    d[a] = l[a];
                }
                shadow = 1;
                orc_slab(o, d, &t, &tf);
                if (!(t < tf)) {
                    for (int ch = 0; ch < 3; ++ch) L[ch] += beta[ch] * (double)po->E[ch] / (4.0 * ORC_PI);
                    new_dir = 1;
                }
            }
        }
        if (new_dir) {
            shadow = 0;
            if (depth >= po->max_depth) return;
            float u1 = (float)orc_rng_u01(seed, 8u, key + i++);
            float u2 = (float)orc_rng_u01(seed, 8u, key + i++);
            float z = 1.0f - 2.0f * u1;
            double rr = sqrt(fmax(0.0, 1.0 - (double)z * (double)z));
            double ph = 2.0 * ORC_PI * (double)u2;
            o[0] = xs[0];
            o[1] = xs[1];
            o[2] = xs[2];
            d[0] = (float)(rr * cos(ph));
            d[1] = (float)(rr * sin(ph));
            d[2] = z;
            orc_slab(o, d, &t, &tf);
            if (!(t < tf)) {
                for (int ch = 0; ch < 3; ++ch) L[ch] += beta[ch] * (double)po->B[ch];
                return;
            }
        }
    }
}

/* opts = { density, light[3], E[3], B[3] } as floats, iopts = { spp,
 * rr_depth, max_depth }; mu (binary32, nullable) with mc_dims, mc_cell. */
int orc_render_pixels_pt(const int32_t* desc, const double* params, const float* cam, const float* lut, int W,
                         int H, uint32_t frame_seed, const int64_t* pix, int64_t n_pix, const int32_t* mc_dims,
                         int mc_cell, const float* mu, const float* fopts, const int32_t* iopts, double* rgba,
                         uint32_t* n_real, uint32_t* n_samp)
{
    orc_model m;
    (void)H;
    if (orc_model_from_desc(desc, &m) || m.width > 1024 || m.n_in > 1024) return -1;
    orc_pt_opts po;
    po.density = fopts[0];
    for (int a = 0; a < 3; ++a) {
        po.light[a] = fopts[1 + a];
        po.E[a] = fopts[4 + a];
        po.B[a] = fopts[7 + a];
    }
    po.spp = iopts[0];
    po.rr_depth = iopts[1];
    po.max_depth = iopts[2];
    if (po.spp < 1 || po.spp > 256 || po.rr_depth < 0 || po.max_depth < 1 || po.max_depth > 1024) return -1;
    const double* Wm = params + m.n_table;
    float l[3], amax = 0.0f;
    orc_unit3(po.light, l);
    for (int i = 0; i < 256; ++i)
        if (lut[4 * i + 3] > amax) amax = lut[4 * i + 3];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t p = pix[q];
        orc_ray r = orc_make_ray(cam, W, (int)(p % W), (int)(p / W), frame_seed, 1.0f);
        double L[3] = {0.0, 0.0, 0.0};
        int hits = 0;
        uint32_t nr = 0, ns = 0;
        for (int sidx = 0; sidx < po.spp; ++sidx) {
            int hit = 0;
            uint64_t key = ((uint64_t)p * (uint64_t)po.spp + (uint64_t)sidx) << 24;
            orc_pt_path(&m, params, Wm, lut, &po, l, amax, mc_dims, mc_cell, mu, (uint64_t)frame_seed, key, r.o, r.d,
                        L, &hit, &ns, &nr);
            hits += hit;
        }
        for (int ch = 0; ch < 3; ++ch) rgba[4 * q + ch] = L[ch] / po.spp;
        rgba[4 * q + 3] = (double)hits / po.spp;
        n_real[q] = nr;
        n_samp[q] = ns;
    }
    return 0;
}

/* thread count of the OpenMP loops from now on (the CPU baseline's
 * single-thread figure) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
