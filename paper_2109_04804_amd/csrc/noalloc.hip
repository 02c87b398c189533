// Context-free evaluation of R1 that allocates no device memory: the 1-D operators and the
// face traces (and, with BR1, the traces of the lifted gradient) live in one file-scope
// device array, `scratch`, of SCRATCH_BYTES.  Each GPU holds its own copy of the array from
// the library's load until the process ends; its device address is looked up once per GPU
// with hipGetSymbolAddress and kept, and only that address is handed to kernels.
//
// Every call on a GPU uses that GPU's one array, which keeps the last call's contents (every
// value a call reads is written by the same call first): calls that overlap on one GPU, on
// different streams or from different host threads, race.
#include "hbpc_internal.hpp"

#include <cstring>
#include <mutex>

static __device__ __align__(256) char scratch[size_t(64) << 20];   // SCRATCH_BYTES

namespace {

constexpr size_t SCRATCH_BYTES = sizeof(scratch);     // 64 MiB per GPU
constexpr size_t BASIS_SLOT = 4096;                  // bytes before the traces (operators: <= 178 doubles)
constexpr int MAX_DEVICES = 64;
constexpr int BASIS_MAX = 184;                        // basis_len for N = 7: 2*8*8 + 6*8 + 2 = 178

std::mutex g_mu;
char* g_scratch[MAX_DEVICES];   // device address of `scratch` on each GPU (null until looked up)

// the operator table travels as a kernel argument, so no host buffer has to outlive the call
struct BasisArg {
    double v[BASIS_MAX];
    int n;
};

__global__ void basis_fill_kernel(double* dst, BasisArg b) {
    const int i = threadIdx.x;
    if (i < b.n) dst[i] = b.v[i];
}

// this GPU's address of `scratch` (null on failure)
char* scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch[dev] = static_cast<char*>(p);
    }
    return g_scratch[dev];
}

// trace values per field: nE * 2d faces * nvar * (N+1)^(d-1) face points
size_t trace_len(const GeomHost& g) {
    size_t nfp = 1;
    for (int m = 0; m + 1 < g.D; ++m) nfp *= (size_t)g.NP;
    return (size_t)g.nE * 2 * g.D * g.NV * nfp;
}

}   // namespace

extern "C" int hbpc_residual1_noalloc(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* params,
                                      const double* w, double* r1) {
    if (!mesh || !params || !w || !r1) return HBPC_ERR_ARG;
    Basis1DHost basis;
    GeomHost g;
    FamilyLauncher launch = nullptr;
    int visc = 0, ns = 0;
    std::string msg;
    const int rc = geom_configure(mesh, N, equation, params, basis, g, launch, visc, ns, msg);
    if (rc != HBPC_OK) return rc;
    if (ns) return HBPC_ERR_UNSUPPORTED;   // the BR2 face gradients need a buffer of their own
    const size_t tsz = trace_len(g);
    if (BASIS_SLOT + tsz * sizeof(double) * (visc ? 2 : 1) > SCRATCH_BYTES) return HBPC_ERR_ARG;
    const std::vector<double> table = basis_table(basis);
    if ((int)table.size() > BASIS_MAX) return HBPC_ERR_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HBPC_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return HBPC_ERR_UNSUPPORTED;
    char* base = scratch_address(dev);
    if (!base) return HBPC_ERR_HIP;
    double* dbasis = reinterpret_cast<double*>(base);
    double* trw = reinterpret_cast<double*>(base + BASIS_SLOT);
    double* qtr = trw + tsz;
    hipStream_t st = static_cast<hipStream_t>(params->stream);

    BasisArg b;
    b.n = (int)table.size();
    for (int i = 0; i < BASIS_MAX; ++i) b.v[i] = i < b.n ? table[i] : 0.0;
    hipLaunchKernelGGL(basis_fill_kernel, dim3(1), dim3(256), 0, st, dbasis, b);
    if (hipGetLastError() != hipSuccess) return HBPC_ERR_HIP;
    g.basis64 = dbasis;
    g.basis32 = nullptr;

    LaunchReq r;
    std::memset(&r, 0, sizeof(r));
    r.stream = st;
    r.op = OPK_TRACE;
    r.fld[0] = w;
    r.out[0] = trw;
    r.col = 1;
    if (launch(g, r, 0) != hipSuccess) return HBPC_ERR_HIP;
    if (visc) {
        std::memset(&r, 0, sizeof(r));
        r.stream = st;
        r.op = OPK_LIFT;
        r.fld[0] = w;
        r.trc[0] = trw;
        r.out[0] = qtr;
        if (launch(g, r, 0) != hipSuccess) return HBPC_ERR_HIP;
    }
    std::memset(&r, 0, sizeof(r));
    r.stream = st;
    r.op = OPK_R1;
    r.fld[0] = w;
    r.trc[0] = trw;
    r.qtr[0] = visc ? qtr : nullptr;
    r.out[0] = r1;
    if (launch(g, r, 0) != hipSuccess) return HBPC_ERR_HIP;
    return HBPC_OK;
}
