// link_probe -- bandwidth of the host link as the served path uses it:
// host-to-device and device-to-host copies between pinned host memory and
// device memory (hipMemcpyAsync on streams of their own), one large copy and
// the same bytes as many event-sized copies, each direction alone and both
// directions at once.  Prints one JSON line (GB/s).
//
// Usage: link_probe [MiB] [event KiB]
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                                  \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) {                                                                   \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                  \
            return 1;                                                                             \
        }                                                                                         \
    } while (0)

int main(int argc, char **argv)
{
    const size_t mib = argc > 1 ? std::strtoul(argv[1], nullptr, 10) : 96;
    const size_t ev_kib = argc > 2 ? std::strtoul(argv[2], nullptr, 10) : 1100;
    const size_t bytes = (mib ? mib : 96) << 20, piece = (ev_kib ? ev_kib : 1100) << 10;
    const int reps = 5;
    char *h_in = nullptr, *h_out = nullptr, *d_in = nullptr, *d_out = nullptr;
    CHECK(hipHostMalloc((void **)&h_in, bytes, hipHostMallocDefault));
    CHECK(hipHostMalloc((void **)&h_out, bytes, hipHostMallocDefault));
    CHECK(hipMalloc((void **)&d_in, bytes));
    CHECK(hipMalloc((void **)&d_out, bytes));
    CHECK(hipMemset(d_out, 0, bytes));
    hipStream_t up, down;
    CHECK(hipStreamCreate(&up));
    CHECK(hipStreamCreate(&down));
    // one pass of each kind: 1 = host to device, 2 = device to host, 3 = both
    // at once; pieces: one copy of `bytes` or copies of `piece` bytes
    auto pass = [&](int dirs, bool pieces) -> hipError_t {
        const size_t step = pieces ? piece : bytes;
        for (size_t at = 0; at < bytes; at += step) {
            const size_t n = bytes - at < step ? bytes - at : step;
            if (dirs & 1) {
                const hipError_t e = hipMemcpyAsync(d_in + at, h_in + at, n, hipMemcpyHostToDevice, up);
                if (e != hipSuccess) return e;
            }
            if (dirs & 2) {
                const hipError_t e = hipMemcpyAsync(h_out + at, d_out + at, n, hipMemcpyDeviceToHost, down);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    double gbs[3][2];
    for (int dirs = 1; dirs <= 3; dirs++)
        for (int pieces = 0; pieces < 2; pieces++) {
            CHECK(pass(dirs, pieces != 0));   // warm-up
            CHECK(hipDeviceSynchronize());
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps; r++) CHECK(pass(dirs, pieces != 0));
            CHECK(hipDeviceSynchronize());
            const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            gbs[dirs - 1][pieces] = (double)bytes * reps / s / 1e9;   // per direction
        }
    std::printf("{\"copy_mib\": %zu, \"piece_kib\": %zu, \"h2d_one_gbs\": %.1f, \"h2d_pieces_gbs\": %.1f, "
                "\"d2h_one_gbs\": %.1f, \"d2h_pieces_gbs\": %.1f, \"both_one_each_gbs\": %.1f, "
                "\"both_pieces_each_gbs\": %.1f}\n",
                bytes >> 20, piece >> 10, gbs[0][0], gbs[0][1], gbs[1][0], gbs[1][1], gbs[2][0], gbs[2][1]);
    (void)hipStreamDestroy(up);
    (void)hipStreamDestroy(down);
    (void)hipFree(d_in);
    (void)hipFree(d_out);
    (void)hipHostFree(h_in);
    (void)hipHostFree(h_out);
    return 0;
}
