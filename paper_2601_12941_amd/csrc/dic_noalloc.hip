// dic_correlate_noalloc: dic_correlate for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Per-frame scratch (deformed coefficients, parent keys,
// frontier lists, wave sizes, seed buffers, seed-search scores, the device
// frame record) comes from one file-scope device array instead of the
// context's grow-only buffers; everything else is the context's, allocated by
// dic_create / dic_set_reference.  The kernels and their order are those of
// dic_correlate, so the results are bitwise the same.
#include "dic_context.h"

#include <mutex>

using namespace dicmi;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // DIC_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;
constexpr int kNoallocMaxSeeds = 64;

// One copy per device, held until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress: kernels and copies take the address
// that call returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

static_assert(sizeof(int32_t) * 3 * kNoallocMaxSeeds + sizeof(FrameState) <= kNoallocStageBytes,
              "pinned staging block too small");

} // namespace

namespace dicmi {

// Device address of this device's scratch array (looked up once per device,
// with the device current).  nullptr on failure.
void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

} // namespace dicmi

extern "C" {

int64_t dic_noalloc_scratch_bytes(void) { return static_cast<int64_t>(kScratchBytes); }

dic_status dic_correlate_noalloc(dic_ctx *c, const dic_image *def, const dic_seed *seeds, int32_t nseeds,
                                 dic_result *out)
{
    if (!c) return DIC_E_INVAL;
    c->err.clear();
    dic_status st = check_correlate_args(c, def, 1, seeds, nseeds, out);
    if (st != DIC_OK) return st;
    if (nseeds > kNoallocMaxSeeds) FAIL(DIC_E_INVAL, "nseeds %d (at most %d without allocation)", nseeds,
                                        kNoallocMaxSeeds);
    HIPCHK(hipSetDevice(c->device));
    unsigned char *base = static_cast<unsigned char *>(c->noalloc_base);
    if (!base) FAIL(DIC_E_DEVICE, "scratch array of device %d not found", c->device);

    // carve the scratch: the same buffers dic_correlate keeps per frame
    const size_t nodes = static_cast<size_t>(c->nodes);
    const size_t esz = c->prm.coef_fp16 ? sizeof(__half) : sizeof(float);
    const size_t side = 2 * static_cast<size_t>(c->prm.seed_radius) + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t o_coef = take(c->coef_elems() * esz);
    const size_t o_pkey = take(sizeof(uint64_t) * nodes);
    const size_t o_l0 = take(sizeof(int32_t) * nodes);
    const size_t o_l1 = take(sizeof(int32_t) * nodes);
    const size_t o_cnt = take(sizeof(int32_t) * (nodes + 2));
    const size_t o_stat = take(sizeof(unsigned long long) * 4);
    const size_t o_sp = take(sizeof(double) * 2 * nseeds);
    const size_t o_sn = take(sizeof(int32_t) * nseeds);
    const size_t o_ctr = take(sizeof(int32_t) * 2 * nseeds);
    const size_t o_z = take(sizeof(double) * nseeds * side * side);
    const size_t o_fr = take(sizeof(FrameState));
    if (off > kScratchBytes)
        FAIL(DIC_E_INVAL, "this reference needs %zu bytes of scratch, above the %zu the allocation-free call holds",
             off, kScratchBytes);

    // host staging in the context's pinned block (no host allocation either)
    int32_t *h_nodes = c->h_noalloc;
    int32_t *h_centre = c->h_noalloc + kNoallocMaxSeeds;
    FrameState *h_frame = reinterpret_cast<FrameState *>(c->h_noalloc + 3 * kNoallocMaxSeeds);
    int nuniq = 0;
    st = snap_frame_seeds(c, seeds, 1, nseeds, h_nodes, h_centre, &nuniq);
    if (st != DIC_OK) return st;
    fill_frame(c, *h_frame, *def, *out, base + o_coef, reinterpret_cast<uint64_t *>(base + o_pkey),
               reinterpret_cast<int32_t *>(base + o_l0), reinterpret_cast<int32_t *>(base + o_l1),
               reinterpret_cast<int32_t *>(base + o_cnt), reinterpret_cast<double *>(base + o_sp),
               reinterpret_cast<int32_t *>(base + o_sn), nuniq,
               reinterpret_cast<unsigned long long *>(base + o_stat));
    return run_frames(c, def, 1, nseeds, h_frame, reinterpret_cast<FrameState *>(base + o_fr), h_nodes, h_centre,
                      reinterpret_cast<int32_t *>(base + o_ctr), reinterpret_cast<double *>(base + o_z), false);
}

} // extern "C"
