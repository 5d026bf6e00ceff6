/*
 * cl_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for the Chung-Lu edge
 * generator of Alam & Khan, "Parallel Algorithms for Generating Random
 * Networks with Given Degree Sequences" (arXiv:1406.1215).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * file; the product path never does.  It shares no code, header or constant
 * table with the HIP implementation: every primitive below is written out
 * here from its published definition.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -shared -fPIC
 * (no contraction: every floating-point operation below is one IEEE-754
 * binary64 operation rounded to nearest-even; fma() appears only where the
 * fixed sampling rule calls for it).  No libm function is used by the sampler.
 *
 * What is computed (Sec. 3, Alg. 1 "Sequential Chung-Lu"): for every source
 * node u of a non-increasing weight vector w, the candidates v > u are visited
 * by geometric skips drawn with the running probability p = min(w_u w_v/S, 1);
 * a visited candidate is kept with probability q/p where q is its own
 * probability.  Where the paper leaves a detail open (random source, uniform
 * mapping, log evaluation, loop exit, splitting of heavy tasks) the reading
 * fixed here is the one every implementation must follow bit for bit:
 *
 *   R1  random source: Philox4x32-10 (Salmon et al., SC'11), counter
 *       (t, k, u, 0), key (seed mod 2^32, seed >> 32); t = draw index inside
 *       task segment k of source u.
 *   R2  uniform in (0,1): U53(x) = (2*(x >> 12) + 1) * 2^-53 of a 64-bit word;
 *       r_skip from words (x1:x0), r_acc from words (x3:x2).
 *   R3  log: own range reduction + fixed atanh series (orc_log / orc_log1m).
 *   R4  skip: delta = floor(LOG(r_skip) / LOG1M(p)); the task ends when the
 *       quotient is not below the number of remaining candidates (this also
 *       covers v >= n, where Alg. 1 would otherwise spin).
 *   R5  accept: r_acc * p < q, the division-free form of r < q/p.
 *   R6  heavy tasks are cut into K_u segments with equal quantised weight mass
 *       (exact integer prefix Q); each segment restarts the memoryless skip
 *       process with its own Philox stream, which leaves the law of the edge
 *       set unchanged (the pairs of different segments are independent).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw, */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 3.2 / Fig. 2). */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u   /* multiplier applied to counter word 0 */
#define PHILOX_MUL_B 0xCD9E8D57u   /* multiplier applied to counter word 2 */
#define PHILOX_WEYL_A 0x9E3779B9u  /* key increment, word 0 (golden ratio) */
#define PHILOX_WEYL_B 0xBB67AE85u  /* key increment, word 1 (sqrt(3)-1)    */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* the key is bumped before rounds 2..10 */
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* R2: a 64-bit word -> double in (0,1).  2*(x>>12)+1 < 2^53 is exact, and the */
/* scaling by 2^-53 is exact, so no rounding happens anywhere.               */
double orc_u53(uint64_t x)
{
    uint64_t odd = ((x >> 12) << 1) | 1u;
    return (double)odd * 0x1p-53;
}

/* ------------------------------------------------------------------------ */
/* R3: logarithms.  log(m) = 2 atanh(s) with s = (m-1)/(m+1), and             */
/* atanh(s)/s = sum_j z^j/(2j+1), z = s^2.  Eleven terms (j = 0..10) suffice  */
/* for |s| <= 0.1716 (the range below): the first dropped term is < 1e-18.    */
/* ------------------------------------------------------------------------ */
static double series_coef(int j) { return 1.0 / (double)(2 * j + 1); }  /* RN(1/(2j+1)) */

double orc_poly(double z)
{
    double acc = series_coef(10);
    for (int j = 9; j >= 0; --j)
        acc = fma(acc, z, series_coef(j));
    return acc;
}

/* the two constants of the range reduction, written from their values */
static double root_two(void) { return 1.41421356237309504880168872420969808; }  /* RN(sqrt 2) */
static double log_two(void)  { return 0.693147180559945309417232121458176568; } /* RN(ln 2)   */

/* natural log of a normal double x in (0, 1]:                               */
/*   x = m 2^e, m in [1,2); if m > RN(sqrt2) use m/2, e+1 so m in (0.707,1.414] */
/*   f = m - 1 (exact), s = f/(2+f), log x = e*RN(ln2) + 2 s POLY(s^2)         */
double orc_log(double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    uint64_t mbits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);
    if (m > root_two()) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double l = (2.0 * s) * orc_poly(z);
    return ((double)e * log_two()) + l;
}

/* log(1 - p) for p in (0,1).  Small p uses log(1-p) = -2 atanh(p/(2-p)) so   */
/* that nothing cancels; otherwise 1 - p is formed and passed to orc_log.    */
double orc_log1m(double p)
{
    if (p < 0.25) {
        double s = p / (2.0 - p);
        double z = s * s;
        return -((2.0 * s) * orc_poly(z));
    }
    return orc_log(1.0 - p);
}

/* ------------------------------------------------------------------------ */
/* Weights, probabilities, segmentation (R6)                                */
/* ------------------------------------------------------------------------ */
#define ORC_OK 0
#define ORC_ERR_INVALID_ARG -1
#define ORC_ERR_UNSORTED -2
#define ORC_ERR_NEGATIVE -3
#define ORC_ERR_NONFINITE -4
#define ORC_ERR_TOO_LARGE -5
#define ORC_ERR_CAPACITY -7

/* Input conditions of Sec. 3: non-negative weights sorted non-increasing,   */
/* S > 0.  Additionally S >= w_0 (so every w_u/S <= 1) and w_0 is either 0   */
/* or not below 2^-960 (so 2^32/w_0 is finite).                              */
int orc_validate(const double* w, uint64_t n, double S)
{
    if (n >= 4294967296ull) return ORC_ERR_TOO_LARGE;
    if (!(S > 0.0) || S > 1.7976931348623157e308) return ORC_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < n; ++i) {
        double x = w[i];
        if (x != x || x > 1.7976931348623157e308 || x < -1.7976931348623157e308) return ORC_ERR_NONFINITE;
    }
    for (uint64_t i = 0; i < n; ++i)
        if (!(w[i] >= 0.0)) return ORC_ERR_NEGATIVE;
    for (uint64_t i = 0; i + 1 < n; ++i)
        if (w[i] < w[i + 1]) return ORC_ERR_UNSORTED;
    if (n > 0) {
        if (w[0] > S) return ORC_ERR_INVALID_ARG;
        if (w[0] > 0.0 && w[0] < 0x1p-960) return ORC_ERR_INVALID_ARG;
    }
    return ORC_OK;
}

/* QSCALE = 2^32 / w_0; q_v = floor(w_v * QSCALE); Q_0 = 0, Q_{v+1} = Q_v + q_v */
/* (all in exact 64-bit integers).  This is the integer counterpart of the    */
/* running sum sigma_u of Eq. 6 (sigma_u ~ Q_u / QSCALE).                     */
double orc_qscale(const double* w, uint64_t n)
{
    if (n == 0 || w[0] == 0.0) return 0.0;
    return 4294967296.0 / w[0];
}

void orc_qscan(const double* w, uint64_t n, double qscale, uint64_t* Q)
{
    Q[0] = 0;
    for (uint64_t v = 0; v < n; ++v) {
        double scaled = w[v] * qscale;
        uint64_t q = (uint64_t)floor(scaled);
        Q[v + 1] = Q[v] + q;
    }
}

/* expected edge count of source u from Eq. 1 / Eq. 6, on the quantised mass: */
/*   e_u = (w_u/S) * sum_{v>u} w_v  ~  (a_u * D_u) / QSCALE,  D_u = Q_n - Q_{u+1} */
double orc_ehat(const double* w, uint64_t n, double S, const uint64_t* Q, double qscale, uint64_t u)
{
    if (qscale == 0.0) return 0.0;
    double a = w[u] / S;
    uint64_t D = Q[n] - Q[u + 1];
    return (a * (double)D) / qscale;
}

/* number of segments of source u: 1 unless e_u > E_SEG, else                 */
/* min(ceil(e_u / E_SEG), n-u-1)                                              */
uint64_t orc_nseg(uint64_t n, uint64_t u, double ehat, double e_seg)
{
    if (!(ehat > e_seg) || u + 2 >= n) return 1;
    uint64_t cap = n - u - 1;                  /* at least 2 here */
    double kd = ceil(ehat / e_seg);
    if (kd >= (double)cap) return cap;
    return (uint64_t)kd;
}

/* first v in [lo, hi] with Q_v >= target (Q non-decreasing; Q_hi >= target) */
static uint64_t q_lower_bound(const uint64_t* Q, uint64_t lo, uint64_t hi, uint64_t target)
{
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (Q[mid] >= target) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* segment starts of source u: b_0 = u+1, b_K = n and, for 0 < k < K,         */
/* b_k = min{ v in [u+1, n] : Q_v - Q_{u+1} >= floor(k D_u / K) }.            */
/* floor(k D / K) is formed exactly as k*(D/K) + (k*(D%K))/K (K < 2^32).       */
void orc_seg_bounds(const uint64_t* Q, uint64_t n, uint64_t u, uint64_t K, uint32_t* b)
{
    uint64_t base = Q[u + 1];
    uint64_t D = Q[n] - base;
    b[0] = (uint32_t)(u + 1);
    for (uint64_t k = 1; k < K; ++k) {
        uint64_t target = k * (D / K) + (k * (D % K)) / K;
        b[k] = (uint32_t)q_lower_bound(Q, u + 1, n, base + target);
    }
    b[K] = (uint32_t)n;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1, the body of the while loop of Create-Edges, restricted to one     */
/* segment [j0, end) of source u (segment index k).  Returns the number of   */
/* accepted edges; writes their v into out (if non-NULL, capacity cap); adds */
/* the number of visited candidates to *ncand (if non-NULL).                 */
/* ------------------------------------------------------------------------ */
static double min1(double x) { return (x < 1.0) ? x : 1.0; }

uint64_t orc_segment(const double* w, double a_u, uint64_t seed,
                     uint32_t u, uint32_t k, uint32_t j0, uint32_t end,
                     uint32_t* out, uint64_t cap, uint64_t* ncand)
{
    uint64_t emitted = 0, visited = 0;
    uint32_t j = j0;
    uint32_t t = 0;
    if (j < end) {
        uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
        double p = min1(a_u * w[j]);
        while (p > 0.0) {
            uint32_t ctr[4] = { t, k, u, 0u }, x[4];
            orc_philox4x32_10(ctr, key, x);
            t = t + 1;
            double r_skip = orc_u53(((uint64_t)x[1] << 32) | x[0]);
            double r_acc  = orc_u53(((uint64_t)x[3] << 32) | x[2]);
            uint32_t delta;
            if (p == 1.0) {
                delta = 0;                      /* Alg. 1: delta <- 0 when p = 1 */
            } else {
                double ratio = orc_log(r_skip) / orc_log1m(p);
                if (!(ratio < (double)(end - j)))
                    break;                      /* the skip leaves the segment */
                delta = (uint32_t)ratio;        /* floor of a value in [0, 2^32) */
            }
            uint32_t v = j + delta;             /* skip delta candidates */
            visited++;
            double q = min1(a_u * w[v]);
            if (r_acc * p < q) {                /* keep (u,v) with probability q/p */
                if (out && emitted < cap) out[emitted] = v;
                emitted++;
            }
            p = q;
            j = v + 1;
            if (j >= end) break;
        }
    }
    if (ncand) *ncand += visited;
    return emitted;
}

/* All segments of source u, in segment order; v of the edges into out. */
uint64_t orc_node(const double* w, uint64_t n, double S, uint64_t seed,
                  const uint64_t* Q, double qscale, double e_seg, uint64_t u,
                  uint32_t* out, uint64_t cap, uint64_t* ncand, uint64_t* nseg_out)
{
    if (u + 1 >= n || qscale == 0.0) {
        if (nseg_out) *nseg_out = 1;
        return 0;
    }
    double a = w[u] / S;
    double eh = orc_ehat(w, n, S, Q, qscale, u);
    uint64_t K = orc_nseg(n, u, eh, e_seg);
    if (nseg_out) *nseg_out = K;
    uint32_t* b = (uint32_t*)malloc((size_t)(K + 1) * sizeof(uint32_t));
    if (!b) return 0;
    orc_seg_bounds(Q, n, u, K, b);
    uint64_t total = 0;
    for (uint64_t k = 0; k < K; ++k) {
        uint64_t room = (out && total < cap) ? cap - total : 0;
        total += orc_segment(w, a, seed, (uint32_t)u, (uint32_t)k, b[k], b[k + 1],
                             out ? out + (total < cap ? total : cap) : NULL, room, ncand);
    }
    free(b);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Position-keyed 64-bit digest of an edge list: sum_i mix(mix(i) ^ (u<<32|v)) */
/* with mix = splitmix64's finaliser (Steele, Lea, Flood, OOPSLA 2014).       */
/* ------------------------------------------------------------------------ */
uint64_t orc_mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_hash_edges(const uint32_t* uv, uint64_t m, uint64_t index_base)
{
    uint64_t h = 0;
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t key = ((uint64_t)uv[2 * i] << 32) | uv[2 * i + 1];
        h += orc_mix64(orc_mix64(index_base + i) ^ key);
    }
    return h;
}

/* ------------------------------------------------------------------------ */
/* Create-Edges(w, S, V) for V = [u_begin, u_end): every edge (u,v), sources */
/* ascending, within a source v ascending.  Two passes (count, then fill at  */
/* the prefix offsets) so sources can run on several threads; the output is  */
/* independent of the thread count.  edges may be NULL (count/hash only).    */
/* Returns m (>= 0) or a negative error code; *hash_out gets the digest.      */
/* ------------------------------------------------------------------------ */
int64_t orc_generate(const double* w, uint64_t n, double S, uint64_t seed,
                     uint64_t u_begin, uint64_t u_end, double e_seg,
                     uint32_t* edges, uint64_t cap, uint64_t* hash_out,
                     uint64_t* ncand_out, int nthreads)
{
    int st = orc_validate(w, n, S);
    if (st != ORC_OK) return st;
    if (u_begin > u_end || u_end > n || !(e_seg > 0.0)) return ORC_ERR_INVALID_ARG;
    if (hash_out) *hash_out = 0;
    if (ncand_out) *ncand_out = 0;
    uint64_t nr = u_end - u_begin;
    if (nr == 0) return 0;
    double qscale = orc_qscale(w, n);
    uint64_t* Q = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
    uint64_t* cnt = (uint64_t*)calloc((size_t)nr + 1, sizeof(uint64_t));
    if (!Q || !cnt) { free(Q); free(cnt); return ORC_ERR_INVALID_ARG; }
    orc_qscan(w, n, qscale, Q);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    uint64_t ncand_total = 0;
    /* pass 1: edge count per source */
#pragma omp parallel for schedule(dynamic, 64) reduction(+:ncand_total)
    for (int64_t r = 0; r < (int64_t)nr; ++r) {
        uint64_t nc = 0;
        cnt[r + 1] = orc_node(w, n, S, seed, Q, qscale, e_seg, u_begin + (uint64_t)r,
                              NULL, 0, &nc, NULL);
        ncand_total += nc;
    }
    for (uint64_t r = 0; r < nr; ++r) cnt[r + 1] += cnt[r];   /* exclusive offsets */
    uint64_t m = cnt[nr];
    if (ncand_out) *ncand_out = ncand_total;
    int over = (edges != NULL && m > cap);
    uint64_t hsum = 0;
    if (!over && (edges != NULL || hash_out != NULL)) {
        /* pass 2: fill (u, v) pairs at their offsets, and the digest */
#pragma omp parallel reduction(+:hsum)
        {
            uint64_t tmp_cap = 1024;
            uint32_t* tmp = (uint32_t*)malloc(tmp_cap * sizeof(uint32_t));
#pragma omp for schedule(dynamic, 64)
            for (int64_t r = 0; r < (int64_t)nr; ++r) {
                uint64_t c = cnt[r + 1] - cnt[r];
                if (c == 0) continue;
                if (c > tmp_cap) {
                    free(tmp);
                    tmp_cap = c;
                    tmp = (uint32_t*)malloc(tmp_cap * sizeof(uint32_t));
                }
                uint64_t u = u_begin + (uint64_t)r;
                orc_node(w, n, S, seed, Q, qscale, e_seg, u, tmp, c, NULL, NULL);
                for (uint64_t i = 0; i < c; ++i) {
                    uint64_t pos = cnt[r] + i;
                    if (edges) {
                        edges[2 * pos] = (uint32_t)u;
                        edges[2 * pos + 1] = tmp[i];
                    }
                    hsum += orc_mix64(orc_mix64(pos) ^ ((u << 32) | tmp[i]));
                }
            }
            free(tmp);
        }
    }
    if (hash_out) *hash_out = hsum;
    free(Q);
    free(cnt);
    if (over) return ORC_ERR_CAPACITY;
    return (int64_t)m;
}

/* ------------------------------------------------------------------------ */
/* Uniform consecutive partition (Sec. 4), computed from its definition.    */
/* Costs are Eq. 2, c_u = e_u + 1, with e_u from Eq. 6 taken on the exact    */
/* quantised mass and kept in fixed point (units of 1/256 edge), so that the */
/* cumulative cost C_u = c_0 + ... + c_u is an exact integer:                */
/*     c_u = floor(256 e_u) + 256,   e_u = (w_u/S) (Q_n - sigma_u - q_u)/QSCALE */
/* Eq. 5: n_i = the smallest u with C_u >= i Z/P, Z = C_{n-1}; with integers  */
/* that is C_u * P >= i * Z (128-bit products).  n_0 = 0, n_P = n.  Alg. 2   */
/* is the parallel way of finding the same bounds; this is the plain one.    */
/* ------------------------------------------------------------------------ */
static uint64_t cost_units(const double* w, uint64_t n, double S, const uint64_t* Q,
                           double qscale, uint64_t u, uint64_t sigma_q, uint64_t q_u)
{
    double e = 0.0;
    if (qscale != 0.0) {
        double a = w[u] / S;
        uint64_t D = Q[n] - sigma_q - q_u;         /* = Q_n - Q_{u+1} */
        e = (a * (double)D) / qscale;
    }
    double scaled = e * 256.0;
    if (scaled > 0x1p40) scaled = 0x1p40;          /* clamp: at most 2^32 edges per source */
    return (uint64_t)floor(scaled) + 256u;
}

int orc_partition(const double* w, uint64_t n, double S, uint64_t P, uint64_t* bounds,
                  uint64_t* total_cost_out)
{
    int st = orc_validate(w, n, S);
    if (st != ORC_OK) return st;
    if (P == 0 || P >= 4294967296ull) return ORC_ERR_INVALID_ARG;
    for (uint64_t k = 0; k <= P; ++k) bounds[k] = n;
    bounds[0] = 0;
    if (total_cost_out) *total_cost_out = 0;
    if (n == 0) return ORC_OK;
    double qscale = orc_qscale(w, n);
    uint64_t* Q = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
    uint64_t* C = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    if (!Q || !C) { free(Q); free(C); return ORC_ERR_INVALID_ARG; }
    orc_qscan(w, n, qscale, Q);
    uint64_t acc = 0;
    for (uint64_t u = 0; u < n; ++u) {             /* C_u, sigma_u = Q_u */
        acc += cost_units(w, n, S, Q, qscale, u, Q[u], Q[u + 1] - Q[u]);
        C[u] = acc;
    }
    uint64_t Z = C[n - 1];
    if (total_cost_out) *total_cost_out = Z;
    /* Eq. 5 for i = 1 .. P-1; C is non-decreasing, so the smallest u moves   */
    /* forward with i and one sweep finds them all                           */
    uint64_t u = 0;
    for (uint64_t i = 1; i < P; ++i) {
        unsigned __int128 target = (unsigned __int128)i * Z;
        while (u < n - 1 && (unsigned __int128)C[u] * P < target) ++u;
        bounds[i] = u;
    }
    bounds[P] = n;
    free(Q); free(C);
    return ORC_OK;
}

/* per-node cost C_u (cumulative, fixed point) for tests of Eq. 4 / Lemma 1 */
int orc_costs(const double* w, uint64_t n, double S, uint64_t* cost)
{
    int st = orc_validate(w, n, S);
    if (st != ORC_OK) return st;
    if (n == 0) return ORC_OK;
    double qscale = orc_qscale(w, n);
    uint64_t* Q = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
    if (!Q) return ORC_ERR_INVALID_ARG;
    orc_qscan(w, n, qscale, Q);
    for (uint64_t u = 0; u < n; ++u)
        cost[u] = cost_units(w, n, S, Q, qscale, u, Q[u], Q[u + 1] - Q[u]);
    free(Q);
    return ORC_OK;
}

/* For exact-law tests on tiny graphs (n <= 11): for seeds seed0 .. seed0 +     */
/* nseeds - 1, the edge set of Create-Edges(w, S, V) as a bit mask over the    */
/* pairs (u,v), u < v, numbered row by row.                                    */
int orc_graph_codes(const double* w, uint64_t n, double S, uint64_t seed0, uint64_t nseeds,
                    double e_seg, uint64_t* codes)
{
    int st = orc_validate(w, n, S);
    if (st != ORC_OK) return st;
    if (n > 11) return ORC_ERR_INVALID_ARG;
    double qscale = orc_qscale(w, n);
    uint64_t Q[12];
    orc_qscan(w, n, qscale, Q);
    uint32_t vs[16];
    for (uint64_t s = 0; s < nseeds; ++s) {
        uint64_t code = 0, base = 0;
        for (uint64_t u = 0; u < n; ++u) {
            uint64_t c = orc_node(w, n, S, seed0 + s, Q, qscale, e_seg, u, vs, 16, NULL, NULL);
            for (uint64_t i = 0; i < c; ++i)
                code |= 1ull << (base + (vs[i] - u - 1));
            base += n - u - 1;
        }
        codes[s] = code;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* S of Alg. 1 for large inputs: the exact sum rounded once to nearest, by   */
/* Shewchuk's error-free accumulation ("Adaptive precision floating-point   */
/* arithmetic", 1997): a list of non-overlapping partials is kept exact with */
/* two-sum; the partials are then added from the largest, with the final    */
/* half-way correction that makes the result correctly rounded.  Returns    */
/* 0 on success, -4 if an intermediate overflows.                            */
/* ------------------------------------------------------------------------ */
int orc_exact_sum(const double* x, uint64_t n, double* out)
{
    size_t cap = 64, np = 0;
    double* p = (double*)malloc(cap * sizeof(double));
    if (!p) return ORC_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < n; ++i) {
        double v = x[i];
        size_t k = 0;
        for (size_t j = 0; j < np; ++j) {
            double y = p[j];
            double a = (fabs(v) < fabs(y)) ? y : v;
            double b = (fabs(v) < fabs(y)) ? v : y;
            double hi = a + b;
            double lo = b - (hi - a);
            if (lo != 0.0) p[k++] = lo;
            v = hi;
        }
        if (v - v != 0.0) { free(p); return ORC_ERR_NONFINITE; }   /* inf: the sum overflowed */
        np = k;
        if (np + 1 > cap) {
            cap *= 2;
            double* q = (double*)realloc(p, cap * sizeof(double));
            if (!q) { free(p); return ORC_ERR_INVALID_ARG; }
            p = q;
        }
        p[np++] = v;
    }
    /* sum the partials from the top; stop at the first inexact addition */
    double hi = 0.0, lo = 0.0;
    size_t j = np;
    if (j > 0) {
        hi = p[--j];
        while (j > 0) {
            double y = p[--j];
            double s = hi + y;
            lo = y - (s - hi);
            hi = s;
            if (lo != 0.0) break;
        }
        /* half-way case: if the remaining partials push past the tie, round
           the other way (the neighbouring partial has the same sign as lo) */
        if (j > 0 && ((lo < 0.0 && p[j - 1] < 0.0) || (lo > 0.0 && p[j - 1] > 0.0))) {
            double y = lo * 2.0;
            double s = hi + y;
            if (y == s - hi) hi = s;
        }
    }
    free(p);
    *out = hi;
    return ORC_OK;
}
