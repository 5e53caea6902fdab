// Images to and from files: parallel positional I/O, O_DIRECT where the
// file system takes it (the image buffers are page aligned), the unaligned
// tail written and read through the page cache. ckpt_dump_file and
// ckpt_restore_file overlap the file I/O with the dump's copy-out and with
// the restore's uploads.
#include <errno.h>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
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

// ------------------------------------------------------------ overlapped file I/O
namespace {

// Whole aligned range [lo, lo + len) of p to or from fd, through an aligned
// bounce buffer when p is pinned host memory (direct I/O cannot address it).
bool piece_io(int fd, uint8_t* p, uint64_t lo, uint64_t len, bool write, uint8_t* bounce) {
    uint8_t* io = bounce ? bounce : p + lo;
    if (bounce && write) memcpy(bounce, p + lo, len);
    uint64_t done = 0;
    while (done < len) {
        const ssize_t r = write ? pwrite(fd, io + done, len - done, (off_t)(lo + done))
                                : pread(fd, io + done, len - done, (off_t)(lo + done));
        if (r < 0 && errno == EINTR) continue;
        if (r <= 0) return false;
        done += (uint64_t)r;
    }
    if (bounce && !write) memcpy(p + lo, bounce, len);
    return true;
}

// The unaligned end [lo, n) of a file through the page cache.
bool tail_io(const char* path, uint8_t* p, uint64_t lo, uint64_t n, bool write) {
    if (lo >= n) return true;
    const int fd = open(path, write ? O_WRONLY : O_RDONLY);
    if (fd < 0) return false;
    bool ok = true;
    uint64_t done = 0;
    while (ok && done < n - lo) {
        const ssize_t r = write ? pwrite(fd, p + lo + done, n - lo - done, (off_t)(lo + done))
                                : pread(fd, p + lo + done, n - lo - done, (off_t)(lo + done));
        if (r < 0 && errno == EINTR) continue;
        if (r <= 0) ok = false;
        else done += (uint64_t)r;
    }
    if (write && ok && fsync(fd) != 0) ok = false;
    close(fd);
    return ok;
}

uint8_t* aligned_buffer() {
    void* q = nullptr;
    return posix_memalign(&q, kAlign, kPiece) == 0 ? static_cast<uint8_t*>(q) : nullptr;
}

// Writes the image of a dump to a file while the dump copies it into host
// memory: each kPiece piece of the file is written as soon as every byte of
// it has been copied (the copies never overlap, so a piece is complete when
// the bytes reported for it add up to kPiece); the pieces holding the header
// and tables, and the last one, once the dump is done.
class FileSink : public PayloadSink {
public:
    FileSink(int fd, bool direct, uint32_t threads, int device)
        : fd_(fd), direct_(direct), device_(device) {
        for (uint32_t i = 0; i < threads; ++i) pool_.emplace_back([this] { work(); });
    }
    ~FileSink() override { end(); }

    void begin(ckpt_image* im) override {
        std::lock_guard<std::mutex> g(mu_);
        im_ = im;
        npieces_ = (im->cap + kPiece - 1) / kPiece;
        got_.reset(new std::atomic<uint64_t>[npieces_]);
        written_.reset(new std::atomic<bool>[npieces_]);
        for (uint64_t k = 0; k < npieces_; ++k) {
            got_[k] = 0;
            written_[k] = false;
        }
    }

    hipError_t issued(hipStream_t s, uint64_t lo, uint64_t hi) override {
        hipEvent_t e;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        if ((r = hipEventRecord(e, s)) != hipSuccess) {
            (void)hipEventDestroy(e);
            return r;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            q_.push_back({e, lo, hi});
        }
        cv_.notify_one();
        return hipSuccess;
    }

    void end() override {
        {
            std::lock_guard<std::mutex> g(mu_);
            closing_ = true;
        }
        cv_.notify_all();
        for (auto& t : pool_) t.join();
        pool_.clear();
    }

    // After a successful dump: the pieces not written yet (header and
    // tables, the last one), then the file is synced. n = image bytes.
    bool finish(const char* path, uint64_t n, uint32_t threads) {
        end();
        if (failed_) return false;
        std::vector<uint64_t> todo;
        const uint64_t aligned = direct_ ? n & ~(kAlign - 1) : n;
        for (uint64_t k = 0; k * kPiece < aligned; ++k)
            if (!written_[k]) todo.push_back(k);
        std::atomic<uint64_t> next{0};
        std::atomic<bool> bad{false};
        auto work = [&]() {
            uint8_t* b = direct_ && im_->pinned ? aligned_buffer() : nullptr;
            if (direct_ && im_->pinned && !b) bad = true;
            for (uint64_t i; !bad && (i = next.fetch_add(1)) < todo.size();) {
                const uint64_t lo = todo[i] * kPiece, len = std::min(kPiece, aligned - lo);
                if (!piece_io(fd_, im_->p, lo, len, true, b)) bad = true;
            }
            free(b);
        };
        std::vector<std::thread> ts;
        for (uint32_t i = 1; i < std::max<uint32_t>(1, threads); ++i) ts.emplace_back(work);
        work();
        for (auto& t : ts) t.join();
        if (bad || !tail_io(path, im_->p, aligned, n, true)) return false;
        return fsync(fd_) == 0;
    }

private:
    struct Item {
        hipEvent_t ev;
        uint64_t lo, hi;
    };
    void work() {
        (void)hipSetDevice(device_);
        uint8_t* bounce = nullptr;
        for (;;) {
            Item it;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return closing_ || !q_.empty(); });
                if (q_.empty()) break;
                it = q_.front();
                q_.pop_front();
            }
            const bool ok = hipEventSynchronize(it.ev) == hipSuccess;
            (void)hipEventDestroy(it.ev);
            if (!ok) failed_ = true;
            if (failed_) continue;
            for (uint64_t k = it.lo / kPiece; k * kPiece < it.hi && k < npieces_; ++k) {
                const uint64_t a = std::max(it.lo, k * kPiece), b = std::min(it.hi, (k + 1) * kPiece);
                if (got_[k].fetch_add(b - a) + (b - a) != kPiece) continue;
                if (direct_ && im_->pinned && !bounce && !(bounce = aligned_buffer())) {
                    failed_ = true;
                    break;
                }
                if (!piece_io(fd_, im_->p, k * kPiece, kPiece, true, direct_ && im_->pinned ? bounce : nullptr))
                    failed_ = true;
                written_[k] = true;
            }
        }
        free(bounce);
    }

    int fd_;
    bool direct_;
    int device_;
    ckpt_image* im_ = nullptr;
    uint64_t npieces_ = 0;
    std::unique_ptr<std::atomic<uint64_t>[]> got_;
    std::unique_ptr<std::atomic<bool>[]> written_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Item> q_;
    bool closing_ = false;
    std::atomic<bool> failed_{false};
    std::vector<std::thread> pool_;
};

// Loads a file into an image piece by piece (threads take pieces in
// increasing order) and lets a restore wait for a prefix of it.
class FileGate : public LoadGate {
public:
    FileGate(int fd, bool direct, const char* path, ckpt_image* im, uint64_t n, uint64_t start, uint32_t threads)
        : fd_(fd), direct_(direct), path_(path), im_(im), n_(n), aligned_(direct ? n & ~(kAlign - 1) : n) {
        npieces_ = (aligned_ + kPiece - 1) / kPiece;
        first_ = std::min<uint64_t>(start / kPiece, npieces_);
        next_ = first_;
        prefix_ = first_;
        done_.assign(npieces_, 0);
        for (uint32_t i = 0; i < std::max<uint32_t>(1, threads); ++i) pool_.emplace_back([this] { work(); });
    }
    ~FileGate() override { stop(); }

    bool wait(uint64_t hi) override {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return failed_ || loaded() >= std::min(hi, n_); });
        return !failed_;
    }

    void stop() {
        stop_ = true;
        for (auto& t : pool_) t.join();
        pool_.clear();
    }

private:
    uint64_t loaded() const {   // under mu_
        if (prefix_ < npieces_) return prefix_ * kPiece;
        return tail_done_ ? n_ : aligned_;
    }
    void work() {
        uint8_t* bounce = direct_ && im_->pinned ? aligned_buffer() : nullptr;
        bool ok = !(direct_ && im_->pinned) || bounce;
        for (;;) {
            uint64_t k;
            {
                std::lock_guard<std::mutex> g(mu_);
                if (!ok) failed_ = true;
                if (failed_ || stop_) break;
                k = next_++;
                if (k >= npieces_) {
                    // the unaligned end, once, by the first thread past the last piece
                    if (k == npieces_ && aligned_ < n_) {
                        ok = tail_io(path_, im_->p, aligned_, n_, false);
                        if (ok) tail_done_ = true;
                        else failed_ = true;
                        cv_.notify_all();
                    } else if (aligned_ == n_) {
                        tail_done_ = true;
                    }
                    break;
                }
            }
            const uint64_t lo = k * kPiece, len = std::min(kPiece, aligned_ - lo);
            ok = piece_io(fd_, im_->p, lo, len, false, bounce);
            std::lock_guard<std::mutex> g(mu_);
            if (!ok) failed_ = true;
            done_[k] = 1;
            while (prefix_ < npieces_ && done_[prefix_]) ++prefix_;
            cv_.notify_all();
        }
        free(bounce);
        std::lock_guard<std::mutex> g(mu_);
        cv_.notify_all();
    }

    int fd_;
    bool direct_;
    const char* path_;
    ckpt_image* im_;
    uint64_t n_, aligned_, npieces_ = 0, first_ = 0, next_ = 0, prefix_ = 0;
    bool tail_done_ = false;
    std::vector<uint8_t> done_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool failed_ = false;
    std::atomic<bool> stop_{false};
    std::vector<std::thread> pool_;
};

void clear_result(ckpt_result* res) {
    if (!res) return;
    memset(res, 0, sizeof(*res));
    res->first_bad_chunk = ~0ull;
}

}  // namespace

extern "C" int ckpt_dump_file(ckpt_ctx* c, const ckpt_alloc_table* table, const ckpt_image* prev, const char* path,
                              uint32_t threads, const ckpt_opts* o, void* stream, ckpt_result* res,
                              ckpt_image** out) {
    clear_result(res);
    if (out) *out = nullptr;
    if (!c || !table || !path) return CKPT_EINVAL;
    if (!threads) threads = 8;
    bool direct = false;
    const int fd = open_file(path, O_WRONLY | O_CREAT | O_TRUNC, &direct);
    if (fd < 0) return CKPT_EIO;
    ckpt_image* im = nullptr;
    int rc;
    {
        FileSink sink(fd, direct, threads, c->device);
        {
            std::lock_guard<std::mutex> g(c->mu);
            rc = dump_impl(c, table, prev, &im, o, stream, res, &sink);
        }
        if (rc == CKPT_OK && !sink.finish(path, im->n, threads)) rc = CKPT_EIO;
    }
    close(fd);
    if (rc != CKPT_OK) {
        if (im) image_release(im);
        unlink(path);
        return rc;
    }
    if (out) *out = im;
    else image_release(im);
    return CKPT_OK;
}

extern "C" int ckpt_restore_file(ckpt_ctx* c, const char* path, uint32_t threads, const ckpt_alloc_table* table,
                                 const ckpt_opts* o, void* stream, ckpt_result* res) {
    clear_result(res);
    if (!c || !path || !table) return CKPT_EINVAL;
    if (!threads) threads = 8;
    struct stat st;
    if (stat(path, &st) != 0) return CKPT_EIO;
    const uint64_t n = (uint64_t)st.st_size;
    if (n < kHeader) return CKPT_ECORRUPT;
    ckpt_image* im = image_new(n);
    if (!im) return CKPT_ENOMEM;
    im->n = n;
    bool direct = false;
    const int fd = open_file(path, O_RDONLY, &direct);
    if (fd < 0) {
        image_release(im);
        return CKPT_EIO;
    }
    // header, then the pieces holding the tables, before the restore starts
    const uint64_t aligned = direct ? n & ~(kAlign - 1) : n;
    uint8_t* bounce = direct && im->pinned ? aligned_buffer() : nullptr;
    int rc = CKPT_OK;
    uint64_t start = std::min(kPiece, aligned);
    if ((direct && im->pinned && !bounce) || (start && !piece_io(fd, im->p, 0, start, false, bounce))) rc = CKPT_EIO;
    if (rc == CKPT_OK && start < kHeader && !tail_io(path, im->p, start, n, false)) rc = CKPT_EIO;
    if (rc == CKPT_OK) {
        const uint8_t* h = im->p;
        const uint32_t flags = get32(h + 12), n_allocs = get32(h + 20);
        const uint64_t n_chunks = get64(h + 24);
        if (n_chunks > (1ull << 40) || n_allocs > (1u << 24)) rc = CKPT_ECORRUPT;
        const uint64_t need = std::min(n, kHeader + tables_len(n_allocs, n_chunks, flags & kFlagCodec));
        while (rc == CKPT_OK && start < std::min(need, aligned)) {
            const uint64_t len = std::min(kPiece, aligned - start);
            if (!piece_io(fd, im->p, start, len, false, bounce)) rc = CKPT_EIO;
            start += len;
        }
        if (rc == CKPT_OK && need > aligned) {
            if (!tail_io(path, im->p, aligned, n, false)) rc = CKPT_EIO;
            start = n;
        }
    }
    free(bounce);
    if (rc == CKPT_OK) {
        FileGate gate(fd, direct, path, im, n, start, threads);
        {
            std::lock_guard<std::mutex> g(c->mu);
            rc = restore_impl(c, im, table, o, stream, res, false, &gate);
        }
        gate.stop();
    }
    close(fd);
    image_release(im);
    return rc;
}
