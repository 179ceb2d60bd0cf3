// The handle behind flapw_handle, and small host helpers shared by the library's host code.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "flapw.h"

namespace flapw {

// A device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= n && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            n = 0;
            if (e != hipSuccess) return e;
        }
        const size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return e;
        }
        n = want;
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

inline long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

constexpr int kRowAlign = 256;      // contraction rows of the work layout are padded to this

}  // namespace flapw

struct flapw_context {
    int device = 0;
    std::string err;
    flapw::DevBuf work;        // P and Q panels of the k-points of one batch
    flapw::DevBuf tmat;        // T of all types (ldt x ldt each)
    flapw::DevBuf tables;      // atoms, types, row weights, Q-kernel tables, repack map
    flapw::DevBuf gaunt;       // Legendre table, quadrature nodes, integrals
    flapw::DevBuf tiles;       // problem descriptors and tile list of a contraction launch
    flapw::DevBuf digits;      // split precision: digit planes and column exponents
    flapw::DevBuf sdesc;       // split precision: descriptors
    flapw::DevBuf leg;         // S through the addition theorem: Khat, radial factors, phases of one k-point
    flapw::DevBuf radial;      // radial setup: meshes, potentials, functions and integral tables
    int s_method = 0;          // flapw_s_method of flapw_hs_generate and flapw_plan_create
    int lnonsph = -1;          // structured T (flapw_set_lnonsph); -1: dense T
    bool inter = false;        // flapw_set_interstitial: generation adds the interstitial terms
    double v_int = 0.0;
    double lattice[9] = {};
    void *blas = nullptr;      // rocblas_handle of flapw_eigensolve (created on first use)
    long long ws_limit = -1;   // flapw_set_workspace_limit: free the work buffers above it after a call
    flapw::DevBuf eig;         // flapw_eigensolve: off-diagonal workspace and status word
    std::vector<unsigned char> host_tables, host_gaunt, host_tiles, host_sdesc;
    std::vector<long long> host_src;
    // tuning (flapw_tune): chosen digit count and tile band per (precision, padded contraction rows,
    // S method, lnonsph)
    struct Tuned {
        int prec;
        long long kp2;
        int s_method;
        int lnonsph;
        int slices;
        int band;
        int chunks;            // modular contraction: 16-row chunks per LDS stage (0: not tuned)
    };
    std::vector<Tuned> tuned;
    // profiling: event pairs per kernel family, recorded while `profiling` is set
    bool profiling = false;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> prof;
    std::vector<hipEvent_t> spare_events;
};

// A captured S/H generation (flapw_plan_create): its own device buffers and the graph.
struct flapw_plan_s {
    flapw_handle h = nullptr;
    flapw::DevBuf work, digits, tmat, tables, gaunt, desc, leg;
    std::vector<unsigned char> h_tables, h_gaunt, h_desc;
    hipGraphExec_t exec = nullptr;
};

namespace flapw {

inline flapw_status fail(flapw_handle h, flapw_status s, const std::string &msg)
{
    if (h) h->err = msg;
    return s;
}

inline flapw_status dev_fail(flapw_handle h, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, e == hipErrorOutOfMemory ? FLAPW_ERR_NOMEM : FLAPW_ERR_DEVICE, m);
}

// Append `count` objects to a byte buffer at a 256-byte aligned offset; returns the offset.
template <class T>
size_t put(std::vector<unsigned char> &buf, const T *src, size_t count)
{
    const size_t off = (size_t)round_up((long long)buf.size(), 256);
    buf.resize(off + sizeof(T) * count);
    if (count) std::memcpy(buf.data() + off, src, sizeof(T) * count);
    return off;
}

// Host-to-device copy of a descriptor buffer (pageable source; the copy is staged before the
// call returns, and the source vector lives in the handle until the next call anyway).
inline flapw_status upload(flapw_handle h, DevBuf &dst, const std::vector<unsigned char> &src, hipStream_t s)
{
    hipError_t e = dst.ensure(src.size());
    if (e != hipSuccess) return dev_fail(h, e, "allocating descriptor buffer");
    e = hipMemcpyAsync(dst.p, src.data(), src.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dev_fail(h, e, "uploading descriptors");
    return FLAPW_OK;
}

// Records an event pair around a launch when profiling is on:  ProfScope p(h, "name", s); launch...
struct ProfScope {
    flapw_handle h;
    hipStream_t s;
    hipEvent_t e1 = nullptr;
    ProfScope(flapw_handle h_, const char *family, hipStream_t s_) : h(h_), s(s_)
    {
        if (!h || !h->profiling) return;
        hipEvent_t e0 = take(), e = take();
        if (!e0 || !e) return;
        (void)hipEventRecord(e0, s);
        e1 = e;
        h->prof.push_back({family, {e0, e1}});
    }
    ~ProfScope()
    {
        if (e1) (void)hipEventRecord(e1, s);
    }
    hipEvent_t take()
    {
        if (!h->spare_events.empty()) {
            hipEvent_t e = h->spare_events.back();
            h->spare_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

// split precision (split.hip)
void split_release(flapw_handle h);
// the eigensolver's rocBLAS handle and workspace (eigen.cpp)
void eigen_release(flapw_handle h);
long long split_bytes(flapw_handle h);

}  // namespace flapw
