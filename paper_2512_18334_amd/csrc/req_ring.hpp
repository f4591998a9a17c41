// req_ring.hpp -- bookkeeping of the serving request ring: byte ranges of
// one device buffer handed out at a moving head and given back in any order.
// Host code only (no device memory is touched here); the caller serialises
// calls.  A piece is taken at the head when it fits between the head and
// the end of the buffer, else at offset 0 when it fits before the oldest
// live piece; the tail is the start of the oldest piece not yet given back.
#pragma once
#include <cstdint>
#include <deque>

namespace vc {

class ReqRing {
  public:
    static constexpr uint64_t ALIGN = 256;

    explicit ReqRing(uint64_t cap = 0) : cap_(cap) {}
    void reset(uint64_t cap) {
        cap_ = cap;
        live_.clear();
        head_ = tail_ = 0;
    }
    uint64_t cap() const { return cap_; }
    size_t live() const { return live_.size(); }

    // a range of at least `bytes` bytes at *at; false (nothing taken) when
    // the ring has no such free range now
    bool take(uint64_t bytes, uint64_t* at) {
        if (bytes == 0 || bytes > cap_) return false;
        bytes = (bytes + ALIGN - 1) & ~(ALIGN - 1);
        if (bytes > cap_) return false;
        uint64_t a;
        if (live_.empty()) {
            head_ = tail_ = 0;
            a = 0;
        } else if (head_ > tail_) {
            // live pieces in [tail, head): room after them, else before
            if (bytes <= cap_ - head_) a = head_;
            else if (bytes <= tail_) a = 0;
            else return false;
        } else {
            // wrapped: the free range is [head, tail)
            if (bytes <= tail_ - head_) a = head_;
            else return false;
        }
        *at = a;
        head_ = a + bytes;
        live_.push_back({a, bytes, false});
        return true;
    }

    // give back the live piece that starts at `at` (unknown offsets are
    // ignored); the tail moves past every piece given back in front of it
    void give(uint64_t at) {
        for (auto& q : live_)
            if (q.at == at && !q.back) {
                q.back = true;
                break;
            }
        while (!live_.empty() && live_.front().back) live_.pop_front();
        if (live_.empty()) head_ = tail_ = 0;
        else tail_ = live_.front().at;
    }

  private:
    struct Piece {
        uint64_t at, bytes;
        bool back;
    };
    uint64_t cap_ = 0, head_ = 0, tail_ = 0;
    std::deque<Piece> live_;
};

}  // namespace vc
