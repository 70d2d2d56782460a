/* Fast CSR assembly of Dirichlet stencil matrices (test-input generator).
 *
 * Same definition as the numpy assembler in sspcg_inputs/__init__.py: for
 * every in-domain neighbour j of cell i the entry is -w_ij with
 * w_ij = 2 k_i k_j / (k_i + k_j) (w = 1 without coefficients); the diagonal is
 * the sum of the neighbour weights in offset order plus k_i for every stencil
 * neighbour outside the domain.  Columns come out sorted because the offsets
 * are passed sorted by linear offset.  Built with -ffp-contract=off so the
 * values equal the numpy ones bit for bit.  Rows are independent, so the
 * z-planes are filled in parallel.
 *
 * inp_scaled_matvec serves the Lanczos interval estimate only (an input of
 * the solver, computed once per workload).
 */
#include <stdint.h>
#include <stdlib.h>

static int in_range(int v, int d, int L) { return v + d >= 0 && v + d < L; }

static int row_count(int z, int y, int x, int Nz, int Ny, int Nx, int K, const int* offs)
{
    int c = 0;
    for (int k = 0; k < K; ++k)
        c += in_range(z, offs[3 * k], Nz) && in_range(y, offs[3 * k + 1], Ny)
             && in_range(x, offs[3 * k + 2], Nx);
    return c;
}

/* Count the nonzeros (returns -1 on bad arguments). */
int64_t inp_stencil_nnz(int Nz, int Ny, int Nx, int K, const int* offs)
{
    if (Nz < 1 || Ny < 1 || Nx < 1 || K < 1) return -1;
    int64_t nnz = 0;
    #pragma omp parallel for reduction(+ : nnz) schedule(static)
    for (int z = 0; z < Nz; ++z)
        for (int y = 0; y < Ny; ++y)
            for (int x = 0; x < Nx; ++x)
                nnz += row_count(z, y, x, Nz, Ny, Nx, K, offs);
    return nnz;
}

/* Fill row_ptr[n+1], col[nnz], val[nnz].  kappa may be NULL (all ones). */
int inp_stencil(int Nz, int Ny, int Nx, int K, const int* offs,
                const double* kappa, int32_t* row_ptr, int32_t* col, double* val)
{
    if (Nz < 1 || Ny < 1 || Nx < 1 || K < 1) return -1;
    const int64_t n = (int64_t)Nz * Ny * Nx;
    /* row lengths, then an exclusive prefix sum */
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < Nz; ++z)
        for (int y = 0; y < Ny; ++y)
            for (int x = 0; x < Nx; ++x) {
                const int64_t i = x + (int64_t)Nx * (y + (int64_t)Ny * z);
                row_ptr[i + 1] = row_count(z, y, x, Nz, Ny, Nx, K, offs);
            }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];

    #pragma omp parallel for schedule(static)
    for (int z = 0; z < Nz; ++z)
        for (int y = 0; y < Ny; ++y)
            for (int x = 0; x < Nx; ++x) {
                const int64_t i = x + (int64_t)Nx * (y + (int64_t)Ny * z);
                int64_t e = row_ptr[i];
                const double ki = kappa ? kappa[i] : 1.0;
                double diag = 0.0;
                int nvalid = 0;
                int64_t diag_pos = -1;
                for (int k = 0; k < K; ++k) {
                    const int dz = offs[3 * k], dy = offs[3 * k + 1], dx = offs[3 * k + 2];
                    if (!(in_range(z, dz, Nz) && in_range(y, dy, Ny) && in_range(x, dx, Nx)))
                        continue;
                    const int64_t j = i + dx + (int64_t)Nx * (dy + (int64_t)Ny * dz);
                    col[e] = (int32_t)j;
                    if (dz == 0 && dy == 0 && dx == 0) {
                        diag_pos = e;
                    } else {
                        double w = 1.0;
                        if (kappa) {
                            const double kj = kappa[j];
                            w = 2.0 * ki * kj / (ki + kj);
                        }
                        val[e] = -w;
                        diag += w;
                        ++nvalid;
                    }
                    ++e;
                }
                const int nmiss = (K - 1) - nvalid;
                diag += (double)nmiss * ki;
                if (diag_pos >= 0) val[diag_pos] = diag;
            }
    return 0;
}

/* w = dh .* (A (dh .* v)), rows in parallel. */
void inp_scaled_matvec(int64_t n, const int32_t* row_ptr, const int32_t* col,
                       const double* val, const double* dh, const double* v, double* w)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            acc += val[e] * (dh[col[e]] * v[col[e]]);
        w[i] = dh[i] * acc;
    }
}

/* d[i] = A_ii (0 where the row stores no diagonal). */
void inp_diagonal(int64_t n, const int32_t* row_ptr, const int32_t* col,
                  const double* val, double* d)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double di = 0.0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col[e] == i) di = val[e];
        d[i] = di;
    }
}
