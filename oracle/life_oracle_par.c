/*
 * Multi-threaded FP64 CPU oracle for the two sparse-Tucker products of LiFE,
 * used to time the CPU baseline and to check whole full-size outputs.
 *
 * TEST INFRASTRUCTURE ONLY.  Like life_oracle.c, nothing in the product path may
 * link, load or call this file; it shares no code, header or table with the HIP
 * library.
 *
 * It computes exactly what life_oracle.c computes (DSC y = M w and WC g = M^T y,
 * eq. 1 with the encoding M_v = D Phi_v of eq. 3, and the transpose product of
 * eq. 6), in double precision, but over its own copies of the nonzeros grouped
 * by voxel (for DSC) and by fascicle (for WC), so that OpenMP threads own whole
 * output entries and no atomics are needed.  The grouping is a stable counting
 * sort, so inside one voxel (one fascicle) the nonzeros keep their input order:
 * every output entry receives the same additions in the same order as in the
 * sequential oracle, and the two agree bit for bit.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t nnz;
    int32_t n_theta, n_voxels, n_fascicles;
    /* grouped by voxel, input order inside a voxel */
    int64_t *vptr;   /* [n_voxels + 1] */
    int16_t *v_atom;
    int32_t *v_fas;
    double *v_phi;
    /* grouped by fascicle, input order inside a fascicle */
    int64_t *fptr;   /* [n_fascicles + 1] */
    int16_t *f_atom;
    int32_t *f_vox;
    double *f_phi;
} oracle_par_t;

static int64_t *group(int64_t nnz, int32_t nkeys, const int32_t *key, int64_t **pos_out)
{
    int64_t *ptr = calloc((size_t)nkeys + 1, sizeof(int64_t));
    int64_t *pos = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!ptr || !pos) { free(ptr); free(pos); return NULL; }
    for (int64_t c = 0; c < nnz; ++c) ++ptr[key[c] + 1];
    for (int32_t k = 0; k < nkeys; ++k) ptr[k + 1] += ptr[k];
    int64_t *next = malloc(sizeof(int64_t) * ((size_t)nkeys + 1));
    if (!next) { free(ptr); free(pos); return NULL; }
    memcpy(next, ptr, sizeof(int64_t) * ((size_t)nkeys + 1));
    for (int64_t c = 0; c < nnz; ++c) pos[next[key[c]]++] = c;   /* stable */
    free(next);
    *pos_out = pos;
    return ptr;
}

void oracle_par_free(oracle_par_t *o)
{
    if (!o) return;
    free(o->vptr); free(o->v_atom); free(o->v_fas); free(o->v_phi);
    free(o->fptr); free(o->f_atom); free(o->f_vox); free(o->f_phi);
    free(o);
}

oracle_par_t *oracle_par_new(int64_t nnz, int32_t n_theta, int32_t n_voxels, int32_t n_fascicles,
                             const int16_t *atom, const int32_t *voxel, const int32_t *fascicle, const double *phi)
{
    oracle_par_t *o = calloc(1, sizeof(oracle_par_t));
    if (!o) return NULL;
    o->nnz = nnz; o->n_theta = n_theta; o->n_voxels = n_voxels; o->n_fascicles = n_fascicles;
    size_t n = (size_t)(nnz > 0 ? nnz : 1);
    int64_t *pos = NULL;
    o->vptr = group(nnz, n_voxels, voxel, &pos);
    o->v_atom = malloc(sizeof(int16_t) * n); o->v_fas = malloc(sizeof(int32_t) * n); o->v_phi = malloc(sizeof(double) * n);
    if (!o->vptr || !o->v_atom || !o->v_fas || !o->v_phi) { free(pos); oracle_par_free(o); return NULL; }
    for (int64_t i = 0; i < nnz; ++i) {
        o->v_atom[i] = atom[pos[i]]; o->v_fas[i] = fascicle[pos[i]]; o->v_phi[i] = phi[pos[i]];
    }
    free(pos);
    pos = NULL;
    o->fptr = group(nnz, n_fascicles, fascicle, &pos);
    o->f_atom = malloc(sizeof(int16_t) * n); o->f_vox = malloc(sizeof(int32_t) * n); o->f_phi = malloc(sizeof(double) * n);
    if (!o->fptr || !o->f_atom || !o->f_vox || !o->f_phi) { free(pos); oracle_par_free(o); return NULL; }
    for (int64_t i = 0; i < nnz; ++i) {
        o->f_atom[i] = atom[pos[i]]; o->f_vox[i] = voxel[pos[i]]; o->f_phi[i] = phi[pos[i]];
    }
    free(pos);
    return o;
}

/* y = M w: each thread owns whole voxels. */
void oracle_par_dsc(const oracle_par_t *o, const double *D, const double *w, double *y)
{
    const int32_t nt = o->n_theta;
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t v = 0; v < o->n_voxels; ++v) {
        double *yv = y + (int64_t)nt * v;
        for (int32_t t = 0; t < nt; ++t) yv[t] = 0.0;
        for (int64_t c = o->vptr[v]; c < o->vptr[v + 1]; ++c) {
            const double s = o->v_phi[c] * w[o->v_fas[c]];
            const double *d = D + (int64_t)nt * o->v_atom[c];
            for (int32_t t = 0; t < nt; ++t) yv[t] += d[t] * s;
        }
    }
}

/* g = M^T y: each thread owns whole fascicles. */
void oracle_par_wc(const oracle_par_t *o, const double *D, const double *y, double *g)
{
    const int32_t nt = o->n_theta;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t f = 0; f < o->n_fascicles; ++f) {
        double acc = 0.0;
        for (int64_t c = o->fptr[f]; c < o->fptr[f + 1]; ++c) {
            const double *d = D + (int64_t)nt * o->f_atom[c];
            const double *yv = y + (int64_t)nt * o->f_vox[c];
            double dot = 0.0;
            for (int32_t t = 0; t < nt; ++t) dot += d[t] * yv[t];
            acc += o->f_phi[c] * dot;
        }
        g[f] = acc;
    }
}

/* Threads an OpenMP parallel region of this library uses. */
int oracle_par_threads(void) { return omp_get_max_threads(); }
