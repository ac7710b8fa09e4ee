// Host-to-device table copies that a captured graph can replay (the class
// is declared with its contract in internal.hpp).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "internal.hpp"

namespace cb {

namespace {
// User-object destructor: runs on a runtime thread after the owning graph
// is destroyed and makes no HIP calls.
void release_block(void* p) { std::free(p); }
}  // namespace

void HostUpload::add(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return;
    if (count_ < (int)(sizeof(items_) / sizeof(items_[0]))) items_[count_] = Item{dst, src, bytes};
    ++count_;
}

cb_status HostUpload::run(hipStream_t st, const char* what) {
    constexpr int kMax = (int)(sizeof(items_) / sizeof(items_[0]));
    if (count_ > kMax) return fail(CB_EINVAL, "%s: %d table copies exceed %d", what, count_, kMax);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t graph = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t ndeps = 0;
    if (hipStreamGetCaptureInfo_v2(st, &cs, &id, &graph, &deps, &ndeps) != hipSuccess)
        return fail(CB_EHIP, "%s: stream capture query failed", what);
    if (cs == hipStreamCaptureStatusInvalidated)
        return fail(CB_EHIP, "%s: the stream's capture has been invalidated", what);
    if (cs == hipStreamCaptureStatusNone) {
        for (int k = 0; k < count_; ++k)
            if (hipMemcpyAsync(items_[k].dst, items_[k].src, items_[k].bytes, hipMemcpyHostToDevice, st) !=
                hipSuccess)
                return fail(CB_EHIP, "%s: table upload failed", what);
        return CB_OK;
    }
    // capturing: one block of copies, owned by the graph
    size_t total = 0;
    for (int k = 0; k < count_; ++k) total += (items_[k].bytes + 63) / 64 * 64;
    char* block = static_cast<char*>(std::malloc(total));
    if (!block) return fail(CB_EHIP, "%s: out of host memory (%zu bytes) for a captured upload", what, total);
    size_t off = 0;
    for (int k = 0; k < count_; ++k) {
        std::memcpy(block + off, items_[k].src, items_[k].bytes);
        off += (items_[k].bytes + 63) / 64 * 64;
    }
    hipUserObject_t obj = nullptr;
    if (hipUserObjectCreate(&obj, block, release_block, 1, hipUserObjectNoDestructorSync) != hipSuccess) {
        std::free(block);
        return fail(CB_EHIP, "%s: cannot create the captured tables' owner", what);
    }
    // the graph takes the only reference: the block lives as long as it
    if (hipGraphRetainUserObject(graph, obj, 1, hipGraphUserObjectMove) != hipSuccess) {
        (void)hipUserObjectRelease(obj, 1);  // frees the block through release_block
        return fail(CB_EHIP, "%s: the captured graph cannot own its tables", what);
    }
    off = 0;
    for (int k = 0; k < count_; ++k) {
        if (hipMemcpyAsync(items_[k].dst, block + off, items_[k].bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return fail(CB_EHIP, "%s: captured table upload failed", what);
        off += (items_[k].bytes + 63) / 64 * 64;
    }
    return CB_OK;
}

}  // namespace cb
