// Generalized Hermitian eigenproblem H c = eps S c of one k-point (section 2.3, eq. matrix_kohnsham),
// the step after the generation in the self-consistency cycle the paper lists.  The dense
// reduction and the tridiagonal eigensolver are rocSOLVER's zhegvd (Cholesky S = U^H U, the
// reduced standard problem U^-H H U^-1, divide and conquer, back-transformation), called on the
// caller's stream through a rocBLAS handle that the library handle owns.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "common.hpp"
#include "context.hpp"

using namespace flapw;

namespace flapw {

void eigen_release(flapw_handle h)
{
    if (h->blas) (void)rocblas_destroy_handle((rocblas_handle)h->blas);
    h->blas = nullptr;
    h->eig.release();
}

}  // namespace flapw

extern "C" flapw_status flapw_eigensolve(flapw_handle h, int n, flapw_z *H, long ldh, flapw_z *S, long lds, double *w,
                                         int vectors, flapw_stream stream)
{
    if (!h) return FLAPW_ERR_ARG;
    if (!H || !S || !w) return fail(h, FLAPW_ERR_ARG, "NULL pointer argument");
    if (n < 1) return fail(h, FLAPW_ERR_ARG, "n must be >= 1");
    if (ldh < n || lds < n) return fail(h, FLAPW_ERR_ARG, "leading dimension < n");
    if (ldh > 0x7fffffffL || lds > 0x7fffffffL) return fail(h, FLAPW_ERR_ARG, "leading dimension beyond 32 bits");
    if (h->device < 0) return fail(h, FLAPW_ERR_DEVICE, "no HIP device");
    hipStream_t s = (hipStream_t)stream;
    if (!h->blas) {
        rocblas_handle bh = nullptr;
        if (rocblas_create_handle(&bh) != rocblas_status_success) return fail(h, FLAPW_ERR_DEVICE, "rocblas_create_handle");
        h->blas = bh;
    }
    rocblas_handle bh = (rocblas_handle)h->blas;
    if (rocblas_set_stream(bh, s) != rocblas_status_success) return fail(h, FLAPW_ERR_DEVICE, "rocblas_set_stream");
    // off-diagonal workspace (n doubles) and the status word
    const size_t ebytes = ((size_t)n * sizeof(double) + 255) / 256 * 256;
    hipError_t e = h->eig.ensure(ebytes + 256);
    if (e != hipSuccess) return dev_fail(h, e, "allocating eigensolver workspace");
    double *E = (double *)h->eig.p;
    rocblas_int *info = (rocblas_int *)((unsigned char *)h->eig.p + ebytes);
    rocblas_status rs;
    {
        ProfScope prof(h, "eigensolve", s);
        rs = rocsolver_zhegvd(bh, rocblas_eform_ax, vectors ? rocblas_evect_original : rocblas_evect_none,
                              rocblas_fill_upper, n, (rocblas_double_complex *)H, (rocblas_int)ldh,
                              (rocblas_double_complex *)S, (rocblas_int)lds, w, E, info);
    }
    if (rs == rocblas_status_memory_error) return fail(h, FLAPW_ERR_NOMEM, "rocsolver_zhegvd: out of device memory");
    if (rs != rocblas_status_success)
        return fail(h, FLAPW_ERR_DEVICE, std::string("rocsolver_zhegvd: ") + rocblas_status_to_string(rs));
    rocblas_int hinfo = 0;
    e = hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(h, e, "reading the eigensolver status");
    if (hinfo > n) return fail(h, FLAPW_ERR_NOT_POSDEF, "S is not positive definite (leading minor " +
                                                            std::to_string(hinfo - n) + ")");
    if (hinfo > 0) return fail(h, FLAPW_ERR_NO_CONVERGENCE, "eigensolver did not converge");
    return FLAPW_OK;
}
