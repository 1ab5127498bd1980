/*
 * CPU oracle of the Hough-transform track finder -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  The product path never calls it and shares no code with
 * it.  It is deliberately plain: one thread, loops in the order of the
 * definition, no blocking, no vectorisation tricks.
 *
 * What it computes (Section 3, the description of the Hough transform): every
 * track hypothesis starts with zero votes; every hit adds one vote to every
 * hypothesis it is compatible with; local maxima of the vote array are then
 * the track candidates.
 *
 * Track model (transverse plane, units cm).  A hypothesis (d0, phi0, kappa)
 * is the circle whose point of closest approach to the origin is
 * P0 = (-d0 sin phi0, d0 cos phi0), moving along (cos phi0, sin phi0) there,
 * with signed curvature kappa.  For a fixed (d0, phi0) and a hit h = (x, y)
 * exactly one kappa puts h on that circle:
 *     u     = y cos(phi0) - x sin(phi0)       (signed offset of h along the
 *                                             normal at P0, plus d0)
 *     kappa = 2 (u - d0) / (r^2 - 2 d0 u + d0^2),   r^2 = x^2 + y^2
 * i.e. twice the offset of h from the tangent line at P0 over the squared
 * chord |h - P0|^2.  At d0 = 0 this is 2 sin(phi_h - phi0) / r.
 *
 * Binning and arithmetic (the paper fixes neither; this is the reading used):
 *   - every operation is one IEEE-754 binary32 operation, round to nearest
 *     even, evaluated in the order C parses the expressions below; no
 *     contraction into FMA (build with -ffp-contract=off), denormals kept;
 *   - the phi0 bin-centre cosines/sines and d0 bin centres are inputs;
 *   - kf = (kappa - kappa_min) * kappa_scale; the vote lands in kappa bin
 *     (int)kf when 0 <= kf < n_kappa; NaN or infinite kf casts no vote;
 *   - a 2D grid is the 3D definition with one d0 bin at d0 = +0.
 *
 * Peak rule (Section 3: track candidates are the local maxima of the votes):
 * a cell with v >= threshold is a candidate when, for every neighbour w at
 * offset o in {-1,0,1}^3 \ {0} (d0, phi0, kappa order), v > w if o is
 * lexicographically negative and v >= w otherwise.  phi0 is periodic; d0 and
 * kappa neighbours outside the grid are ignored.  Candidates are sorted by
 * votes descending, then cell index ascending, cell = (l*n_phi + j)*n_kappa + k.
 *
 * Straight tracks: hough_oracle_vote_straight below (the two-parameter
 * family); its peaks are the peak rule above on a (1, n_phi, n_d0) array.
 *
 * Forward-hemisphere option (forward != 0; an addition, not the paper's
 * method): a hit votes for a phi0 bin only when it lies ahead of P0 along
 * (cos phi0, sin phi0), i.e. ahead = x cos(phi0) + y sin(phi0) > 0, one
 * binary32 operation each in that order (P0 itself is orthogonal to the
 * direction, so the test does not involve d0).  Every hit is compatible with
 * two directions of travel through it; the cut keeps the one moving away from
 * the origin and drops the mirror solution (for a prompt track, the peak at
 * phi0 + pi with the opposite curvature).  A hit exactly abreast (ahead == 0)
 * does not vote.
 *
 * Hit association (Section 3 reads each track candidate as the hits that
 * made it): hough_oracle_associate below; its reading is stated above it.
 *
 * Displaced vertices (Section 5): hough_oracle_vertex_vote and
 * hough_oracle_vertex_peaks below take the candidates to a binned (x, y)
 * vertex grid; their reading is stated above them.
 *
 * Parity pins live in tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Vote every hit into the accumulator (Section 3).  acc is int64 [n_d0][n_phi][n_kappa],
 * overwritten.  d0 == NULL means a 2D grid (n_d0 must be 1, d0 = +0).  forward != 0 applies
 * the forward-hemisphere option.  Returns the number of votes cast, or -1 on invalid
 * arguments. */
int64_t hough_oracle_vote(int64_t n_hits, const float *x, const float *y,
                          int32_t n_d0, const float *d0,
                          int32_t n_phi, const float *cos_phi, const float *sin_phi,
                          int32_t n_kappa, float kappa_min, float kappa_scale,
                          int32_t forward, int64_t *acc)
{
    if (n_hits < 0 || n_d0 < 1 || n_phi < 1 || n_kappa < 1 || !acc)
        return -1;
    if (d0 == NULL && n_d0 != 1)
        return -1;
    int64_t cells = (int64_t)n_d0 * n_phi * n_kappa;
    memset(acc, 0, (size_t)cells * sizeof(int64_t));
    const float n_kappa_f = (float)n_kappa;
    int64_t votes = 0;
    for (int64_t i = 0; i < n_hits; ++i) {
        float xi = x[i];
        float yi = y[i];
        float r2 = xi * xi + yi * yi;
        for (int32_t l = 0; l < n_d0; ++l) {
            float d = d0 ? d0[l] : 0.0f;
            for (int32_t j = 0; j < n_phi; ++j) {
                float c = cos_phi[j];
                float s = sin_phi[j];
                if (forward) {
                    float ahead = xi * c + yi * s;
                    if (!(ahead > 0.0f))
                        continue;
                }
                float u = yi * c - xi * s;
                float num = 2.0f * (u - d);
                float den = r2 - 2.0f * d * u + d * d;
                float kappa = num / den;
                float kf = (kappa - kappa_min) * kappa_scale;
                if (kf >= 0.0f && kf < n_kappa_f) {
                    int32_t k = (int32_t)kf;
                    acc[((int64_t)l * n_phi + j) * n_kappa + k] += 1;
                    votes += 1;
                }
            }
        }
    }
    return votes;
}

/* Straight tracks (Section 3: a straight line needs two parameters, the
 * kappa = 0 family): the hypothesis (phi0, d0) is the line through
 * P0 = (-d0 sin phi0, d0 cos phi0) along (cos phi0, sin phi0).  A hit lies on
 * it when u = y cos(phi0) - x sin(phi0) equals d0, so for every phi0 bin it
 * votes d0 bin (int)fd, fd = (u - d0_min) * d0_scale, when 0 <= fd < n_d0
 * (binary32 operations in this order).  forward != 0 applies the
 * forward-hemisphere option.  acc is int64 [n_phi][n_d0], overwritten;
 * cell = j * n_d0 + k.  Returns the number of votes. */
int64_t hough_oracle_vote_straight(int64_t n_hits, const float *x, const float *y,
                                   int32_t n_phi, const float *cos_phi, const float *sin_phi,
                                   int32_t n_d0, float d0_min, float d0_scale, int32_t forward,
                                   int64_t *acc)
{
    if (n_hits < 0 || n_phi < 1 || n_d0 < 1 || !acc)
        return -1;
    memset(acc, 0, (size_t)n_phi * (size_t)n_d0 * sizeof(int64_t));
    const float n_d0_f = (float)n_d0;
    int64_t votes = 0;
    for (int64_t i = 0; i < n_hits; ++i) {
        const float xh = x[i];
        const float yh = y[i];
        for (int32_t j = 0; j < n_phi; ++j) {
            if (forward) {
                float fwd = xh * cos_phi[j] + yh * sin_phi[j];
                if (!(fwd > 0.0f))
                    continue;
            }
            float along = yh * cos_phi[j] - xh * sin_phi[j];
            float fd = (along - d0_min) * d0_scale;
            if (fd >= 0.0f && fd < n_d0_f) {
                acc[(int64_t)j * n_d0 + (int32_t)fd] += 1;
                votes += 1;
            }
        }
    }
    return votes;
}

typedef struct {
    int64_t votes;
    int64_t cell;
} oracle_cand;

static int cand_order(const void *pa, const void *pb)
{
    const oracle_cand *a = (const oracle_cand *)pa;
    const oracle_cand *b = (const oracle_cand *)pb;
    if (a->votes != b->votes)
        return a->votes > b->votes ? -1 : 1;
    if (a->cell != b->cell)
        return a->cell < b->cell ? -1 : 1;
    return 0;
}

/* Is cell (l, j, k) with value v a local maximum under the tie rule above? */
static int is_local_max(int32_t n_d0, int32_t n_phi, int32_t n_kappa, const int64_t *acc,
                        int32_t l, int32_t j, int32_t k, int64_t v)
{
    for (int od = -1; od <= 1; ++od) {
        for (int op = -1; op <= 1; ++op) {
            for (int ok = -1; ok <= 1; ++ok) {
                if (od == 0 && op == 0 && ok == 0)
                    continue;
                int32_t ll = l + od;
                int32_t kk = k + ok;
                if (ll < 0 || ll >= n_d0 || kk < 0 || kk >= n_kappa)
                    continue;
                int32_t jj = j + op;
                if (jj < 0)
                    jj += n_phi;
                if (jj >= n_phi)
                    jj -= n_phi;
                int64_t w = acc[((int64_t)ll * n_phi + jj) * n_kappa + kk];
                int negative = od != 0 ? od < 0 : (op != 0 ? op < 0 : ok < 0);
                if (negative ? !(v > w) : !(v >= w))
                    return 0;
            }
        }
    }
    return 1;
}

/* Threshold + local-maximum search + sort (Section 3).  Writes the first min(n_found, cap)
 * candidates to out_votes/out_cell (either may be NULL when cap == 0).  Returns n_found,
 * or -1 on invalid arguments / allocation failure. */
int64_t hough_oracle_peaks(int32_t n_d0, int32_t n_phi, int32_t n_kappa, const int64_t *acc,
                           int64_t threshold, int64_t cap, int64_t *out_votes, int64_t *out_cell)
{
    if (n_d0 < 1 || n_phi < 3 || n_kappa < 1 || !acc || cap < 0)
        return -1;
    int64_t n_found = 0;
    int64_t room = 1024;
    oracle_cand *list = (oracle_cand *)malloc((size_t)room * sizeof(oracle_cand));
    if (!list)
        return -1;
    for (int32_t l = 0; l < n_d0; ++l) {
        for (int32_t j = 0; j < n_phi; ++j) {
            for (int32_t k = 0; k < n_kappa; ++k) {
                int64_t cell = ((int64_t)l * n_phi + j) * n_kappa + k;
                int64_t v = acc[cell];
                if (v < threshold)
                    continue;
                if (!is_local_max(n_d0, n_phi, n_kappa, acc, l, j, k, v))
                    continue;
                if (n_found == room) {
                    room *= 2;
                    oracle_cand *grown = (oracle_cand *)realloc(list, (size_t)room * sizeof(oracle_cand));
                    if (!grown) {
                        free(list);
                        return -1;
                    }
                    list = grown;
                }
                list[n_found].votes = v;
                list[n_found].cell = cell;
                n_found += 1;
            }
        }
    }
    qsort(list, (size_t)n_found, sizeof(oracle_cand), cand_order);
    int64_t n_out = n_found < cap ? n_found : cap;
    for (int64_t i = 0; i < n_out; ++i) {
        out_votes[i] = list[i].votes;
        out_cell[i] = list[i].cell;
    }
    free(list);
    return n_found;
}

/*
 * Displaced-vertex second transform (Section 5: a second Hough transform of
 * the first one's result finds the vertices; a vertex V is the sinusoid
 * d0 = V_y cos(phi0) - V_x sin(phi0) in the (phi0, d0) plane).  Reading:
 * every first-transform candidate with votes >= track_threshold is the
 * straight line through P0 = (-d0 sin phi0, d0 cos phi0) along (cos phi0,
 * sin phi0), i.e. the vertices V with V_y c - V_x s = d0, using the bin
 * centres of its cell.  It votes into a binned (x, y) vertex grid once per
 * column when |c| >= |s| (the line's y at each column centre) and once per
 * row otherwise (its x at each row centre), every operation one binary32
 * operation in the order written:
 *     column ix:  y = (d0 + x_centre[ix] * s) / c,  fy = (y - y_min) * y_scale,
 *                 vote (ix, (int)fy) when 0 <= fy < n_y;
 *     row iy:     x = (y_centre[iy] * c - d0) / s,  fx = (x - x_min) * x_scale,
 *                 vote ((int)fx, iy) when 0 <= fx < n_x.
 * vacc is int64 [n_x][n_y], overwritten; vertex cell = ix * n_y + iy.
 * Returns the number of votes, or -1 on invalid arguments.
 */
int64_t hough_oracle_vertex_vote(int64_t n_cands, const int64_t *cand_votes, const int64_t *cand_cell,
                                 int64_t track_threshold,
                                 int32_t n_d0, const float *d0, int32_t n_phi, const float *cos_phi,
                                 const float *sin_phi, int32_t n_kappa,
                                 int32_t n_x, const float *x_centre, float x_min, float x_scale,
                                 int32_t n_y, const float *y_centre, float y_min, float y_scale,
                                 int64_t *vacc)
{
    if (n_cands < 0 || n_d0 < 1 || n_phi < 1 || n_kappa < 1 || n_x < 1 || n_y < 1 || !vacc)
        return -1;
    if (d0 == NULL && n_d0 != 1)
        return -1;
    memset(vacc, 0, (size_t)n_x * (size_t)n_y * sizeof(int64_t));
    const int64_t track_cells = (int64_t)n_d0 * n_phi * n_kappa;
    const float n_x_f = (float)n_x;
    const float n_y_f = (float)n_y;
    int64_t votes = 0;
    for (int64_t i = 0; i < n_cands; ++i) {
        if (cand_votes[i] < track_threshold)
            continue;
        const int64_t cell = cand_cell[i];
        if (cell < 0 || cell >= track_cells)
            return -1;
        const int32_t l = (int32_t)(cell / ((int64_t)n_phi * n_kappa));
        const int32_t j = (int32_t)((cell / n_kappa) % n_phi);
        const float dt = d0 ? d0[l] : 0.0f;     /* the track's d0 */
        const float c = cos_phi[j];
        const float s = sin_phi[j];
        if (fabsf(c) >= fabsf(s)) {
            for (int32_t ix = 0; ix < n_x; ++ix) {
                float t = x_centre[ix] * s;
                float num = dt + t;
                float yv = num / c;
                float fy = (yv - y_min) * y_scale;
                if (fy >= 0.0f && fy < n_y_f) {
                    vacc[(int64_t)ix * n_y + (int32_t)fy] += 1;
                    votes += 1;
                }
            }
        } else {
            for (int32_t iy = 0; iy < n_y; ++iy) {
                float t = y_centre[iy] * c;
                float num = t - dt;
                float xv = num / s;
                float fx = (xv - x_min) * x_scale;
                if (fx >= 0.0f && fx < n_x_f) {
                    vacc[(int64_t)(int32_t)fx * n_y + iy] += 1;
                    votes += 1;
                }
            }
        }
    }
    return votes;
}

/* Vertex candidates: the peak rule above on the (x, y) grid, neither axis
 * periodic (neighbours outside are ignored), offsets ordered (dx, dy); sorted
 * by votes descending then cell ascending.  Writes the first min(n_found, cap);
 * returns n_found, or -1 on invalid arguments / allocation failure. */
int64_t hough_oracle_vertex_peaks(int32_t n_x, int32_t n_y, const int64_t *vacc, int64_t threshold,
                                  int64_t cap, int64_t *out_votes, int64_t *out_cell)
{
    if (n_x < 1 || n_y < 1 || !vacc || cap < 0)
        return -1;
    int64_t n_found = 0;
    int64_t room = 256;
    oracle_cand *list = (oracle_cand *)malloc((size_t)room * sizeof(oracle_cand));
    if (!list)
        return -1;
    for (int32_t ix = 0; ix < n_x; ++ix) {
        for (int32_t iy = 0; iy < n_y; ++iy) {
            const int64_t val = vacc[(int64_t)ix * n_y + iy];
            if (val < threshold)
                continue;
            int keep = 1;
            for (int dx = -1; dx <= 1 && keep; ++dx) {
                for (int dy = -1; dy <= 1; ++dy) {
                    if (dx == 0 && dy == 0)
                        continue;
                    const int32_t xx = ix + dx;
                    const int32_t yy = iy + dy;
                    if (xx < 0 || xx >= n_x || yy < 0 || yy >= n_y)
                        continue;
                    const int64_t w = vacc[(int64_t)xx * n_y + yy];
                    const int negative = dx != 0 ? dx < 0 : dy < 0;
                    if (negative ? !(val > w) : !(val >= w)) {
                        keep = 0;
                        break;
                    }
                }
            }
            if (!keep)
                continue;
            if (n_found == room) {
                room *= 2;
                oracle_cand *grown = (oracle_cand *)realloc(list, (size_t)room * sizeof(oracle_cand));
                if (!grown) {
                    free(list);
                    return -1;
                }
                list = grown;
            }
            list[n_found].votes = val;
            list[n_found].cell = (int64_t)ix * n_y + iy;
            n_found += 1;
        }
    }
    qsort(list, (size_t)n_found, sizeof(oracle_cand), cand_order);
    const int64_t n_out = n_found < cap ? n_found : cap;
    for (int64_t i = 0; i < n_out; ++i) {
        out_votes[i] = list[i].votes;
        out_cell[i] = list[i].cell;
    }
    free(list);
    return n_found;
}

/*
 * Hit association (Section 3: a track candidate is a local maximum of the
 * votes, made by the hits compatible with it).  Reading: hit h belongs to
 * candidate C = (lc, jc, kc) when h casts a vote into some cell of C's
 * neighbourhood, the cells (lc + dl, jc + dj, kc + dk) with dl, dj, dk in
 * {-1, 0, 1} -- dj modulo n_phi, dl and dk inside the grid, dl = 0 for a 2D
 * or straight grid -- i.e. the same 3x3(x3) window as the peak rule.  The
 * vote is the one of hough_oracle_vote (curved, family 0) or
 * hough_oracle_vote_straight (family 1), with the forward option when
 * forward != 0, recomputed here per (hit, slice, row).  Only candidates with
 * votes >= min_votes take part.  Writes the pairs (candidate index, hit
 * index) in candidate order, hits ascending within a candidate: the first
 * min(n_pairs, cap).  Returns n_pairs, or -1 on invalid arguments.
 */
static int assoc_bin(float hx, float hy, float hr2, int32_t family, int32_t forward, float dl0,
                     float cj, float sj, float kmin, float kscale, int32_t nk, int32_t *bin)
{
    if (forward) {
        float front = hx * cj + hy * sj;
        if (!(front > 0.0f))
            return 0;
    }
    float off = hy * cj - hx * sj;
    float frac;
    if (family == 1) {
        frac = (off - kmin) * kscale;
    } else {
        float twice = 2.0f * (off - dl0);
        float chord2 = hr2 - 2.0f * dl0 * off + dl0 * dl0;
        float curv = twice / chord2;
        frac = (curv - kmin) * kscale;
    }
    if (frac >= 0.0f && frac < (float)nk) {
        *bin = (int32_t)frac;
        return 1;
    }
    return 0;
}

int64_t hough_oracle_associate(int64_t n_hits, const float *x, const float *y,
                               int32_t n_d0, const float *d0, int32_t n_phi, const float *cos_phi,
                               const float *sin_phi, int32_t n_kappa, float kappa_min, float kappa_scale,
                               int32_t family, int32_t forward,
                               int64_t n_cands, const int64_t *cand_votes, const int64_t *cand_cell,
                               int64_t min_votes, int64_t cap, int64_t *out_cand, int64_t *out_hit)
{
    if (n_hits < 0 || n_d0 < 1 || n_phi < 1 || n_kappa < 1 || n_cands < 0 || cap < 0)
        return -1;
    if ((d0 == NULL && n_d0 != 1) || (family != 0 && family != 1) || (family == 1 && d0 != NULL))
        return -1;
    const int64_t cells = (int64_t)n_d0 * n_phi * n_kappa;
    int64_t n_pairs = 0;
    for (int64_t c = 0; c < n_cands; ++c) {
        if (cand_votes[c] < min_votes)
            continue;
        const int64_t cell = cand_cell[c];
        if (cell < 0 || cell >= cells)
            return -1;
        const int32_t lc = (int32_t)(cell / ((int64_t)n_phi * n_kappa));
        const int32_t jc = (int32_t)((cell / n_kappa) % n_phi);
        const int32_t kc = (int32_t)(cell % n_kappa);
        for (int64_t h = 0; h < n_hits; ++h) {
            const float hx = x[h];
            const float hy = y[h];
            const float hr2 = hx * hx + hy * hy;
            int member = 0;
            for (int dl = -1; dl <= 1 && !member; ++dl) {
                const int32_t ll = lc + dl;
                if (ll < 0 || ll >= n_d0)
                    continue;
                const float dl0 = d0 ? d0[ll] : 0.0f;
                for (int dj = -1; dj <= 1 && !member; ++dj) {
                    const int32_t jj = (jc + dj + n_phi) % n_phi;
                    int32_t k;
                    if (assoc_bin(hx, hy, hr2, family, forward, dl0, cos_phi[jj], sin_phi[jj],
                                  kappa_min, kappa_scale, n_kappa, &k) && k >= kc - 1 && k <= kc + 1)
                        member = 1;
                }
            }
            if (!member)
                continue;
            if (n_pairs < cap) {
                out_cand[n_pairs] = c;
                out_hit[n_pairs] = h;
            }
            n_pairs += 1;
        }
    }
    return n_pairs;
}
