// Images to and from files: parallel positional I/O, O_DIRECT where the
// file system takes it (the image buffers are page aligned), the unaligned
// tail written and read through the page cache.
#include <errno.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/mickpt.h"
#include "runtime.h"

using namespace mk;

namespace {

constexpr uint64_t kAlign = 4096;
constexpr uint64_t kPiece = 64ull << 20;

// [0, n) of p to or from fd in kPiece pieces over `threads` threads. With
// `bounce` every piece goes through a page-aligned heap buffer of the
// thread: pinned host memory is a driver mapping, which direct I/O cannot
// address.
bool parallel_io(int fd, uint8_t* p, uint64_t n, bool write, uint32_t threads, bool bounce) {
    std::atomic<uint64_t> next{0};
    std::atomic<bool> failed{false};
    auto work = [&]() {
        uint8_t* buf = nullptr;
        if (bounce) {
            void* q = nullptr;
            if (posix_memalign(&q, kAlign, kPiece) != 0) {
                failed = true;
                return;
            }
            buf = static_cast<uint8_t*>(q);
        }
        for (;;) {
            const uint64_t lo = next.fetch_add(1) * kPiece;
            if (lo >= n || failed.load()) break;
            const uint64_t len = std::min(kPiece, n - lo);
            uint8_t* io = bounce ? buf : p + lo;
            if (bounce && write) memcpy(buf, p + lo, len);
            uint64_t done = 0;
            while (done < len) {
                const ssize_t r = write ? pwrite(fd, io + done, len - done, (off_t)(lo + done))
                                        : pread(fd, io + done, len - done, (off_t)(lo + done));
                if (r < 0 && errno == EINTR) continue;
                if (r <= 0) {
                    failed = true;
                    break;
                }
                done += (uint64_t)r;
            }
            if (failed.load()) break;
            if (bounce && !write) memcpy(p + lo, buf, len);
        }
        free(buf);
    };
    const uint32_t nt = std::max<uint32_t>(1, std::min<uint64_t>(threads, (n + kPiece - 1) / kPiece));
    std::vector<std::thread> pool;
    for (uint32_t i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    return !failed.load();
}

// O_DIRECT when the file system accepts it
int open_file(const char* path, int flags, bool* direct) {
    int fd = open(path, flags | O_DIRECT, 0644);
    *direct = fd >= 0;
    if (fd < 0 && errno == EINVAL) fd = open(path, flags, 0644);
    return fd;
}

}  // namespace

extern "C" int ckpt_image_save(const ckpt_image* img, const char* path, uint32_t threads) {
    if (!img || !path) return CKPT_EINVAL;
    if (!threads) threads = 8;
    const uint64_t n = img->n;
    bool direct = false;
    const int fd = open_file(path, O_WRONLY | O_CREAT | O_TRUNC, &direct);
    if (fd < 0) return CKPT_EIO;
    // the page-aligned prefix (O_DIRECT needs aligned offsets, lengths and buffers)
    const uint64_t head = direct ? n & ~(kAlign - 1) : n;
    bool ok = parallel_io(fd, img->p, head, true, threads, direct && img->pinned);
    if (ok && head < n) {
        const int fd2 = open(path, O_WRONLY);
        ok = fd2 >= 0;
        uint64_t done = 0;
        while (ok && done < n - head) {
            const ssize_t r = pwrite(fd2, img->p + head + done, n - head - done, (off_t)(head + done));
            if (r < 0 && errno == EINTR) continue;
            if (r <= 0) ok = false;
            else done += (uint64_t)r;
        }
        if (fd2 >= 0) {
            if (fsync(fd2) != 0) ok = false;
            close(fd2);
        }
    }
    if (ok && fsync(fd) != 0) ok = false;
    close(fd);
    return ok ? CKPT_OK : CKPT_EIO;
}

extern "C" int ckpt_image_load(const char* path, uint32_t threads, ckpt_image** out) {
    if (!path || !out) return CKPT_EINVAL;
    *out = nullptr;
    if (!threads) threads = 8;
    struct stat st;
    if (stat(path, &st) != 0) return CKPT_EIO;
    const uint64_t n = (uint64_t)st.st_size;
    ckpt_image* im = image_new(n);
    if (!im) return CKPT_ENOMEM;
    bool direct = false;
    const int fd = open_file(path, O_RDONLY, &direct);
    if (fd < 0) {
        image_release(im);
        return CKPT_EIO;
    }
    const uint64_t head = direct ? n & ~(kAlign - 1) : n;
    bool ok = parallel_io(fd, im->p, head, false, threads, direct && im->pinned);
    close(fd);
    if (ok && head < n) {
        const int fd2 = open(path, O_RDONLY);
        ok = fd2 >= 0;
        uint64_t done = 0;
        while (ok && done < n - head) {
            const ssize_t r = pread(fd2, im->p + head + done, n - head - done, (off_t)(head + done));
            if (r < 0 && errno == EINTR) continue;
            if (r <= 0) ok = false;
            else done += (uint64_t)r;
        }
        if (fd2 >= 0) close(fd2);
    }
    if (!ok) {
        image_release(im);
        return CKPT_EIO;
    }
    ImageView v;
    const int rc = parse_image(im->p, n, &v, true);
    if (rc) {
        image_release(im);
        return rc;
    }
    im->n = n;
    *out = im;
    return CKPT_OK;
}
